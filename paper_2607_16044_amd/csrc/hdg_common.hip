// Facet initialisation, the HDG-MX lifting of the mixed variables and the
// SDIRK stage right-hand side.
//
// Lifting (Sec. 3.5, eq. bilinear_form_hdg_mixed, mixed rows): the mixed
// equations are affine in Q = (eps11, eps12, eps22, phi1, phi2) with the mass
// matrix as coefficient, so Q(U, Uhat) = -M_Q^{-1} l(U, Uhat) with
//   l_eps[zeta] = int_T u . div(zeta - tr(zeta)/3 I) - int_dT uhat . (zeta - tr(zeta)/3 I) n
//   l_phi[vphi] = int_T theta div(vphi)              - int_dT thetahat vphi . n
// tested with zeta = E11 phi_n, (E12 + E21) phi_n, E22 phi_n and vphi = e_d phi_n.
// M_Q is diagonal (Gauss-Legendre nodal basis), the (E12 + E21) row carrying a
// factor 2 because eps : zeta counts the off-diagonal entry twice.
#include "ctx.h"

namespace imex {

// element trace at facet node m of local face f (l_b(xi_m) = delta_bm on the nodal basis)
template <int K>
__device__ inline double trace_at_node(const BasisTable& T, int f, int m, const double* u) {
  constexpr int NP = K + 1;
  const int s = f & 1;
  double r = 0.0;
  if (f < 2) {
#pragma unroll
    for (int a = 0; a < NP; ++a) r += T.LE[s][a] * u[a + NP * m];
  } else {
#pragma unroll
    for (int b = 0; b < NP; ++b) r += T.LE[s][b] * u[m + NP * b];
  }
  return r;
}

template <int K>
__global__ void init_facets_kernel(DeviceMesh m, DeviceHDG h, const double* __restrict__ U,
                                   double* __restrict__ Uhat) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * 4 * NP) return;
  const int mnode = t % NP, v = (t / NP) % 4, hf = t / (4 * NP);
  int e[2], f[2];
  int nexp = 0;
  for (int s = 0; s < 2; ++s) {
    e[s] = h.hf_elem[2 * hf + s];
    f[s] = h.hf_face[2 * hf + s];
    if (e[s] >= 0 && !m.imp[e[s]]) ++nexp;
  }
  double acc = 0.0;
  int cnt = 0;
  for (int s = 0; s < 2; ++s) {
    if (e[s] < 0) continue;
    if (nexp > 0 && m.imp[e[s]]) continue;      // interface facet: explicit trace only
    acc += trace_at_node<K>(*m.tab, f[s], mnode, U + (size_t)e[s] * 4 * NN + v * NN);
    ++cnt;
  }
  Uhat[t] = acc / cnt;
}

template <int K>
__global__ void __launch_bounds__(256) lift_mixed_kernel(DeviceMesh m, DeviceHDG h, Gas g,
                                                         const double* __restrict__ U,
                                                         const double* __restrict__ Uhat, double* __restrict__ Q) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  __shared__ double sP[NQV][3];      // u, v, theta at volume points (times w |J|)
  __shared__ double sH[4][NQ][3];    // uhat, vhat, thetahat at face points (times w ds)
  __shared__ double sU[4 * NN];
  const int p = blockIdx.x;
  const int e = h.im_list[p];
  const BasisTable& tb = *m.tab;
  const int tid = threadIdx.x;
  for (int i = tid; i < 4 * NN; i += blockDim.x) sU[i] = U[(size_t)e * 4 * NN + i];
  __syncthreads();
  const double hx = m.hx[e], hy = m.hy[e];
  for (int qv = tid; qv < NQV; qv += blockDim.x) {
    const int qi = qv % NQ, qj = qv / NQ;
    double W[4] = {0, 0, 0, 0};
    for (int b = 0; b < NP; ++b)
      for (int a = 0; a < NP; ++a) {
        const double ph = tb.L[qi][a] * tb.L[qj][b];
#pragma unroll
        for (int v = 0; v < 4; ++v) W[v] += ph * sU[v * NN + a + NP * b];
      }
    const Prim<double> P = primitives(W, g);
    const double w = tb.W[qi] * tb.W[qj] * hx * hy * 0.25;
    sP[qv][0] = w * P.u;
    sP[qv][1] = w * P.v;
    sP[qv][2] = w * P.theta;
  }
  for (int i = tid; i < 4 * NQ; i += blockDim.x) {
    const int f = i / NQ, q = i % NQ;
    const int hf = h.efacet[4 * p + f];
    double W[4] = {0, 0, 0, 0};
    for (int mm = 0; mm < NP; ++mm) {
      const double ps = tb.L[q][mm];
#pragma unroll
      for (int v = 0; v < 4; ++v) W[v] += ps * Uhat[((size_t)hf * 4 + v) * NP + mm];
    }
    const Prim<double> P = primitives(W, g);
    const double w = tb.W[q] * ((f < 2) ? 0.5 * hy : 0.5 * hx);
    sH[f][q][0] = w * P.u;
    sH[f][q][1] = w * P.v;
    sH[f][q][2] = w * P.theta;
  }
  __syncthreads();
  for (int n = tid; n < NN; n += blockDim.x) {
    const int a = n % NP, b = n / NP;
    double l[5] = {0, 0, 0, 0, 0};
    const double sx = 2.0 / hx, sy = 2.0 / hy;
    for (int qj = 0; qj < NQ; ++qj)
      for (int qi = 0; qi < NQ; ++qi) {
        const int qv = qi + NQ * qj;
        const double px = tb.D[qi][a] * tb.L[qj][b] * sx;
        const double py = tb.L[qi][a] * tb.D[qj][b] * sy;
        const double u = sP[qv][0], v = sP[qv][1], th = sP[qv][2];
        l[0] += (2.0 / 3.0) * u * px - (1.0 / 3.0) * v * py;
        l[1] += u * py + v * px;
        l[2] += -(1.0 / 3.0) * u * px + (2.0 / 3.0) * v * py;
        l[3] += th * px;
        l[4] += th * py;
      }
    for (int f = 0; f < 4; ++f) {
      const int s = f & 1;
      const double nx = (f == 0) ? -1.0 : (f == 1 ? 1.0 : 0.0);
      const double ny = (f == 2) ? -1.0 : (f == 3 ? 1.0 : 0.0);
      for (int q = 0; q < NQ; ++q) {
        const double ph = (f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b];
        const double u = sH[f][q][0], v = sH[f][q][1], th = sH[f][q][2];
        l[0] -= ph * ((2.0 / 3.0) * u * nx - (1.0 / 3.0) * v * ny);
        l[1] -= ph * (u * ny + v * nx);
        l[2] -= ph * (-(1.0 / 3.0) * u * nx + (2.0 / 3.0) * v * ny);
        l[3] -= ph * th * nx;
        l[4] -= ph * th * ny;
      }
    }
    const double mass = tb.NW[a] * tb.NW[b] * hx * hy * 0.25;
    const double fac[5] = {1.0, 2.0, 1.0, 1.0, 1.0};
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) Q[(size_t)e * 5 * NN + cc * NN + n] = -l[cc] / (fac[cc] * mass);
  }
}

// rhs = M U_n on implicit elements (the remaining terms are added by axpy)
template <int K>
__global__ void mass_rhs_kernel(DeviceMesh m, DeviceHDG h, const double* __restrict__ Un, double* __restrict__ rhs) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_im * 4 * NN) return;
  const int r = t % (4 * NN);
  const int e = h.im_list[t / (4 * NN)];
  const int n = r % NN;
  const BasisTable& tb = *m.tab;
  const double mass = tb.NW[n % NP] * tb.NW[n / NP] * m.hx[e] * m.hy[e] * 0.25;
  const size_t idx = (size_t)e * 4 * NN + r;
  rhs[idx] = mass * Un[idx];
}

// Stage predictor on the implicit rows: a <- Y, Y <- a + c (a - P), P <- a
template <int K>
__global__ void extrapolate_implicit_kernel(DeviceHDG h, double c, double* __restrict__ Y, double* __restrict__ P) {
  constexpr int NN = (K + 1) * (K + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_im * 4 * NN) return;
  const size_t idx = (size_t)h.im_list[t / (4 * NN)] * 4 * NN + t % (4 * NN);
  const double a = Y[idx];
  Y[idx] = a + c * (a - P[idx]);
  P[idx] = a;
}

__global__ void extrapolate_kernel(int n, double c, double* __restrict__ Y, double* __restrict__ P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double a = Y[t];
  Y[t] = a + c * (a - P[t]);
  P[t] = a;
}

// rhs += b dts_e R on the rows of implicit elements
template <int K>
__global__ void rhs_accumulate_kernel(DeviceMesh m, DeviceHDG h, double b, const double* __restrict__ R,
                                      double* __restrict__ rhs) {
  constexpr int NN = (K + 1) * (K + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_im * 4 * NN) return;
  const int e = h.im_list[t / (4 * NN)];
  const size_t idx = (size_t)e * 4 * NN + t % (4 * NN);
  rhs[idx] += b * elem_dt(m, e) * R[idx];
}

// out += a f_e(n) in over the selected rows: rows 0 all, 1 explicit, 2 implicit elements;
// f = 1 (fac 0), the nodal mass (1), dts_e / mass (2) or dts_e (3)
template <int K>
__global__ void rows_axpy_kernel(DeviceMesh m, int rows, int fac, double a, const double* __restrict__ in,
                                 double* __restrict__ out) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * 4 * NN) return;
  const int e = t / (4 * NN), n = t % NN;
  if ((rows == 1 && m.imp[e]) || (rows == 2 && !m.imp[e])) return;
  double f = 1.0;
  if (fac) {
    const BasisTable& tb = *m.tab;
    const double mass = tb.NW[n % NP] * tb.NW[n / NP] * m.hx[e] * m.hy[e] * 0.25;
    f = fac == 1 ? mass : (fac == 2 ? elem_dt(m, e) / mass : elem_dt(m, e));
  }
  out[t] += a * f * in[t];
}

#define IMEX_DISPATCH_K(KV, ...)                                \
  switch (KV) {                                                 \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;       \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;       \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;       \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;       \
    default: return hipErrorInvalidValue;                       \
  }

hipError_t launch_init_facets(const imex_ctx* c, const double* U, double* Uhat) {
  const int n = c->n_hf * 4 * c->NP;
  if (n == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(init_facets_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                           c->dmesh(), c->dhdg(), U, Uhat));
  return hipGetLastError();
}

hipError_t launch_lift_mixed(const imex_ctx* c, const double* U, const double* Uhat, double* Q) {
  if (c->n_im == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(lift_mixed_kernel<KK>, dim3(c->n_im), dim3(64), 0, c->stream, c->dmesh(),
                                           c->dhdg(), c->gas, U, Uhat, Q));
  return hipGetLastError();
}

hipError_t launch_extrapolate(const imex_ctx* c, double coef, double* Y, double* Yp, double* Uhat, double* Hp) {
  const int n = c->n_im * 4 * c->NN;
  if (n == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(extrapolate_implicit_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0,
                                           c->stream, c->dhdg(), coef, Y, Yp));
  const int nh = c->n_hf * 4 * c->NP;
  hipLaunchKernelGGL(extrapolate_kernel, dim3((nh + 255) / 256), dim3(256), 0, c->stream, nh, coef, Uhat, Hp);
  return hipGetLastError();
}

hipError_t launch_rhs_accumulate(const imex_ctx* c, double b, const double* R, double* rhs) {
  const int n = c->n_im * 4 * c->NN;
  if (n == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(rhs_accumulate_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0,
                                           c->stream, c->dmesh(), c->dhdg(), b, R, rhs));
  return hipGetLastError();
}

hipError_t launch_rows_axpy(const imex_ctx* c, int rows, int fac, double a, const double* in, double* out) {
  const int n = c->E * 4 * c->NN;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(rows_axpy_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                           c->dmesh(), rows, fac, a, in, out));
  return hipGetLastError();
}

hipError_t launch_mass_rhs(const imex_ctx* c, const double* Un, double* rhs) {
  const int n = c->n_im * 4 * c->NN;
  if (n == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(mass_rhs_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                           c->dmesh(), c->dhdg(), Un, rhs));
  return hipGetLastError();
}

}  // namespace imex
