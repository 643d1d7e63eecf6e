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

// Transpose of init_facets_kernel for the sides on local face fpass:
// Ub[e] += (trace_f)^T Uhatbar[hf] / cnt.  An element has one face fpass, so within a
// pass every element node has at most one writer; the four passes run in stream order.
template <int K>
__global__ void init_facets_vjp_kernel(DeviceMesh m, DeviceHDG h, int fpass, const double* __restrict__ Hb,
                                       double* __restrict__ Ub) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * 2 * 4 * NN) return;
  const int n = t % NN, v = (t / NN) % 4, s = (t / (4 * NN)) % 2, hf = t / (8 * NN);
  const int e = h.hf_elem[2 * hf + s];
  if (e < 0 || h.hf_face[2 * hf + s] != fpass) return;
  int nexp = 0;
  for (int q = 0; q < 2; ++q) {
    const int eq = h.hf_elem[2 * hf + q];
    if (eq >= 0 && !m.imp[eq]) ++nexp;
  }
  if (nexp > 0 && m.imp[e]) return;                // interface facet: explicit trace only
  int cnt = 0;
  for (int q = 0; q < 2; ++q) {
    const int eq = h.hf_elem[2 * hf + q];
    if (eq >= 0 && !(nexp > 0 && m.imp[eq])) ++cnt;
  }
  const int a = n % NP, b = n / NP;
  const double* hb = Hb + ((size_t)hf * 4 + v) * NP;
  // x faces (0, 1) interpolate along a at face node b; y faces (2, 3) along b at node a
  const double coef = fpass < 2 ? m.tab->LE[fpass & 1][a] * hb[b] : m.tab->LE[fpass & 1][b] * hb[a];
  Ub[((size_t)e * 4 + v) * NN + n] += coef / cnt;
}

// Wall shear of the HDG-MX region: per implicit element, the integral over its adiabatic
// wall faces of 2 mu eps_12 = mu (du/dy + dv/dx), with eps_12 the lifted mixed variable
// Q_1 traced onto the face (Sec. 3.5: the stored strain components).
template <int K>
__global__ void wall_shear_kernel(DeviceMesh m, DeviceHDG h, double mu, const double* __restrict__ Q,
                                  double* __restrict__ part) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= h.n_im) return;
  const int e = h.im_list[p];
  const BasisTable& tb = *m.tab;
  const double* q1 = Q + ((size_t)e * 5 + 1) * NN;
  double acc = 0.0;
  for (int f = 0; f < 4; ++f) {
    if (h.face_kind[4 * p + f] != FK_WALL) continue;
    const int s = f & 1;
    const double wl = (f < 2) ? 0.5 * m.hy[e] : 0.5 * m.hx[e];
    for (int q = 0; q < NQ; ++q) {
      double val = 0.0;
      for (int b = 0; b < NP; ++b)
        for (int a = 0; a < NP; ++a)
          val += ((f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b]) * q1[a + NP * b];
      acc += tb.W[q] * wl * val;
    }
  }
  part[p] = 2.0 * mu * acc;
}

// Qbar = scale * d(wall shear)/dQ: component 1 of implicit elements with wall faces (the
// rest of Qb is left as it is)
template <int K>
__global__ void wall_shear_qbar_kernel(DeviceMesh m, DeviceHDG h, double scale, double* __restrict__ Qb) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_im * NN) return;
  const int p = t / NN, n = t % NN, a = n % NP, b = n / NP;
  const int e = h.im_list[p];
  const BasisTable& tb = *m.tab;
  double acc = 0.0;
  for (int f = 0; f < 4; ++f) {
    if (h.face_kind[4 * p + f] != FK_WALL) continue;
    const int s = f & 1;
    const double wl = (f < 2) ? 0.5 * m.hy[e] : 0.5 * m.hx[e];
    for (int q = 0; q < NQ; ++q)
      acc += tb.W[q] * wl * ((f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b]);
  }
  Qb[((size_t)e * 5 + 1) * NN + n] = scale * acc;
}

// Partial sums (one per block of 256 threads) of a . b for the parameter adjoint:
// kind 0 all element rows; kind 1 implicit rows, each element weighted by its instance
// time-step scale when scaled != 0; kind 2 facet shares: a is a facet vector, b holds
// per-implicit-element facet rows [p][face][v][m], summed as a[facet of face] . b[p][face].
template <int K>
__global__ void __launch_bounds__(256) param_dot_kernel(DeviceMesh m, DeviceHDG h, int E, int kind, int scaled,
                                                        const double* __restrict__ a, const double* __restrict__ b,
                                                        double* __restrict__ part) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NFF = 4 * NP, NF = 4 * NFF;
  __shared__ double red4[4];
  const long long n = kind == 0 ? (long long)E * NU : (long long)h.n_im * (kind == 1 ? NU : NF);
  double acc = 0.0;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
    if (kind == 0) {
      acc += a[t] * b[t];
    } else if (kind == 1) {
      const int p = (int)(t / NU), i = (int)(t % NU), e = h.im_list[p];
      const size_t gi = (size_t)e * NU + i;
      acc += a[gi] * b[gi] * (scaled ? elem_dt(m, e) : 1.0);
    } else {
      const int p = (int)(t / NF), r = (int)(t % NF), f = r / NFF, j = r % NFF;
      acc += a[(size_t)h.efacet[4 * p + f] * NFF + j] * b[t];
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red4[0] + red4[1] + red4[2] + red4[3];
}

// <lamhat, dh/dp> along a far-field direction u_inf + p du: u_inf enters the HDG facet
// rows only on far-field facets, h = int (A^+(Uhat)(Uhat - U) - A^-(Uhat)(Uhat - u_inf)) psi
// (App. B.2.1), whose derivative is int A^-(Uhat) du psi, exactly; the element rows do
// not depend on u_inf.  lamhat is laid out as the facet unknowns.  Per-block partials.
struct HDir4 { double v[4]; };

template <int K>
__global__ void __launch_bounds__(256) hdg_param_dot_kernel(DeviceMesh m, DeviceHDG h, Gas g, HDir4 du,
                                                            const double* __restrict__ H,
                                                            const double* __restrict__ lam, double* __restrict__ part) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NFF = 4 * NP;
  __shared__ double red[4];
  const BasisTable& tb = *m.tab;
  double acc = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < h.n_im * 4 * NQ; t += gridDim.x * blockDim.x) {
    const int q = t % NQ, f = (t / NQ) % 4, pp = t / (4 * NQ);
    if (h.face_kind[4 * pp + f] != FK_FARFIELD) continue;
    const int e = h.im_list[pp];
    const size_t fo = (size_t)h.efacet[4 * pp + f] * NFF;
    double Wh[4], lq[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int mm = 0; mm < NP; ++mm) {
        a += tb.L[q][mm] * H[fo + v * NP + mm];
        b += tb.L[q][mm] * lam[fo + v * NP + mm];
      }
      Wh[v] = a;
      lq[v] = b;
    }
    const double nx = (f == 0) ? -1.0 : (f == 1 ? 1.0 : 0.0), ny = (f == 2) ? -1.0 : (f == 3 ? 1.0 : 0.0);
    double am[4];
    char_apply(Wh, du.v, nx, ny, -1, g, am);
    const double w = tb.W[q] * ((f < 2) ? 0.5 * m.hy[e] : 0.5 * m.hx[e]);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc += w * am[v] * lq[v];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
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
    // the quadrature loops stay rolled: unrolled, the table reads of all 49 points are
    // hoisted into registers and spill
#pragma unroll 1
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
#pragma unroll 1
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

// Reverse mode of the lifting Q = Q(U, Uhat) above: given Qbar [e][5][NN] on implicit
// elements, adds the adjoint of U to Ubar (implicit rows) and writes this element's
// share of the facet adjoint, Hb[p][f][v][m] (summed over both sides by
// facet_gather_kernel).  l_c[n] = -fac_c mass_n Q_c[n] is linear in the primitives
// (u, v, theta) at the volume points (weights w dphi_n/dx_d) and at the face points
// (weights -w phi_n n_d); the primitives' Jacobians come from dual numbers.
template <int K>
__global__ void __launch_bounds__(64) lift_vjp_kernel(DeviceMesh m, DeviceHDG h, Gas g, const double* __restrict__ U,
                                                      const double* __restrict__ Uhat, const double* __restrict__ Qb,
                                                      double* __restrict__ Ub, double* __restrict__ Hb) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  __shared__ double sU[4 * NN];
  __shared__ double lb[5][NN];
  __shared__ double sWb[NQV][4];
  __shared__ double sHb[4][NQ][4];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int e = h.im_list[p];
  const BasisTable& tb = *m.tab;
  const double hx = m.hx[e], hy = m.hy[e], sx = 2.0 / hx, sy = 2.0 / hy, jac = 0.25 * hx * hy;
  const double fac[5] = {1.0, 2.0, 1.0, 1.0, 1.0};
  for (int i = tid; i < 4 * NN; i += blockDim.x) sU[i] = U[(size_t)e * 4 * NN + i];
  for (int i = tid; i < 5 * NN; i += blockDim.x) {
    const int c = i / NN, n = i % NN;
    const double mass = tb.NW[n % NP] * tb.NW[n / NP] * jac;
    lb[c][n] = -Qb[(size_t)e * 5 * NN + i] / (fac[c] * mass);
  }
  __syncthreads();
  using D4 = Dual<4>;
  for (int qv = tid; qv < NQV; qv += blockDim.x) {
    const int qi = qv % NQ, qj = qv / NQ;
    double W[4] = {0, 0, 0, 0}, pb[3] = {0, 0, 0};
    const double w = tb.W[qi] * tb.W[qj] * jac;
#pragma unroll 1
    for (int b = 0; b < NP; ++b)
      for (int a = 0; a < NP; ++a) {
        const int n = a + NP * b;
        const double ph = tb.L[qi][a] * tb.L[qj][b];
        const double px = w * tb.D[qi][a] * tb.L[qj][b] * sx, py = w * tb.L[qi][a] * tb.D[qj][b] * sy;
#pragma unroll
        for (int v = 0; v < 4; ++v) W[v] += ph * sU[v * NN + n];
        pb[0] += lb[0][n] * (2.0 / 3.0) * px + lb[1][n] * py - lb[2][n] * (1.0 / 3.0) * px;
        pb[1] += -lb[0][n] * (1.0 / 3.0) * py + lb[1][n] * px + lb[2][n] * (2.0 / 3.0) * py;
        pb[2] += lb[3][n] * px + lb[4][n] * py;
      }
    D4 Wd[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) { Wd[v] = D4(W[v]); Wd[v].d[v] = 1.0; }
    const Prim<D4> P = primitives(Wd, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) sWb[qv][v] = pb[0] * P.u.d[v] + pb[1] * P.v.d[v] + pb[2] * P.theta.d[v];
  }
  for (int i = tid; i < 4 * NQ; i += blockDim.x) {
    const int f = i / NQ, q = i % NQ, s = f & 1;
    const int hf = h.efacet[4 * p + f];
    const double nx = (f == 0) ? -1.0 : (f == 1 ? 1.0 : 0.0);
    const double ny = (f == 2) ? -1.0 : (f == 3 ? 1.0 : 0.0);
    const double w = tb.W[q] * ((f < 2) ? 0.5 * hy : 0.5 * hx);
    double W[4] = {0, 0, 0, 0};
    for (int mm = 0; mm < NP; ++mm)
#pragma unroll
      for (int v = 0; v < 4; ++v) W[v] += tb.L[q][mm] * Uhat[((size_t)hf * 4 + v) * NP + mm];
    double pb[3] = {0, 0, 0};
#pragma unroll 1
    for (int b = 0; b < NP; ++b)
      for (int a = 0; a < NP; ++a) {
        const int n = a + NP * b;
        const double ph = -w * ((f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b]);
        pb[0] += ph * (lb[0][n] * (2.0 / 3.0) * nx + lb[1][n] * ny - lb[2][n] * (1.0 / 3.0) * nx);
        pb[1] += ph * (-lb[0][n] * (1.0 / 3.0) * ny + lb[1][n] * nx + lb[2][n] * (2.0 / 3.0) * ny);
        pb[2] += ph * (lb[3][n] * nx + lb[4][n] * ny);
      }
    D4 Wd[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) { Wd[v] = D4(W[v]); Wd[v].d[v] = 1.0; }
    const Prim<D4> P = primitives(Wd, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) sHb[f][q][v] = pb[0] * P.u.d[v] + pb[1] * P.v.d[v] + pb[2] * P.theta.d[v];
  }
  __syncthreads();
  for (int i = tid; i < 16 * NP; i += blockDim.x) {
    const int f = i / (4 * NP), v = (i / NP) % 4, mm = i % NP;
    double acc = 0.0;
    for (int q = 0; q < NQ; ++q) acc += tb.L[q][mm] * sHb[f][q][v];
    Hb[(size_t)p * 16 * NP + i] = acc;
  }
  for (int i = tid; i < 4 * NN; i += blockDim.x) {
    const int v = i / NN, n = i % NN, a = n % NP, b = n / NP;
    double acc = 0.0;
    for (int qj = 0; qj < NQ; ++qj)
      for (int qi = 0; qi < NQ; ++qi) acc += tb.L[qi][a] * tb.L[qj][b] * sWb[qi + NQ * qj][v];
    Ub[(size_t)e * 4 * NN + i] += acc;
  }
}

// out[F][v][m] += sum over the implicit sides T of F of Hb[T][face of F][v][m]
template <int K>
__global__ void facet_gather_kernel(DeviceHDG h, const double* __restrict__ Hb, double* __restrict__ out) {
  constexpr int NFF = 4 * (K + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * NFF) return;
  const int hf = t / NFF, j = t % NFF;
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * hf + s];
    if (pe < 0) continue;
    acc += Hb[((size_t)pe * 4 + h.hf_face[2 * hf + s]) * NFF + j];
  }
  out[t] += acc;
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

hipError_t launch_init_facets_vjp(const imex_ctx* c, const double* Hb, double* Ub) {
  const int n = c->n_hf * 2 * 4 * c->NN;
  if (n == 0) return hipSuccess;
  for (int f = 0; f < 4; ++f)
    IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(init_facets_vjp_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0,
                                             c->stream, c->dmesh(), c->dhdg(), f, Hb, Ub));
  return hipGetLastError();
}

hipError_t launch_param_dot(const imex_ctx* c, int kind, int scaled, const double* a, const double* b, double* part,
                            int nblk) {
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(param_dot_kernel<KK>, dim3(nblk), dim3(256), 0, c->stream, c->dmesh(),
                                           c->dhdg(), c->E, kind, scaled, a, b, part));
  return hipGetLastError();
}

hipError_t launch_hdg_param_dot(const imex_ctx* c, const double* du, const double* H, const double* lam, double* part,
                                int nblk) {
  HDir4 d{{du[0], du[1], du[2], du[3]}};
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(hdg_param_dot_kernel<KK>, dim3(nblk), dim3(256), 0, c->stream,
                                           c->dmesh(), c->dhdg(), c->gas, d, H, lam, part));
  return hipGetLastError();
}

hipError_t launch_wall_shear(const imex_ctx* c, const double* Q, double* part) {
  if (c->n_im == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(wall_shear_kernel<KK>, dim3((c->n_im + 63) / 64), dim3(64), 0, c->stream,
                                           c->dmesh(), c->dhdg(), c->gas.mu, Q, part));
  return hipGetLastError();
}

hipError_t launch_wall_shear_qbar(const imex_ctx* c, double scale, double* Qb) {
  const int n = c->n_im * c->NN;
  if (n == 0) return hipSuccess;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(wall_shear_qbar_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0,
                                           c->stream, c->dmesh(), c->dhdg(), scale, Qb));
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

hipError_t launch_lift_vjp(const imex_ctx* c, const double* U, const double* Uhat, const double* Qb, double* Ub,
                           double* Hb, double* Uhatbar) {
  if (c->n_im == 0) return hipSuccess;
  const int nh = c->n_hf * 4 * c->NP;
  IMEX_DISPATCH_K(c->K, {
    hipLaunchKernelGGL(lift_vjp_kernel<KK>, dim3(c->n_im), dim3(64), 0, c->stream, c->dmesh(), c->dhdg(), c->gas, U,
                       Uhat, Qb, Ub, Hb);
    hipLaunchKernelGGL(facet_gather_kernel<KK>, dim3((nh + 255) / 256), dim3(256), 0, c->stream, c->dhdg(), Hb,
                       Uhatbar);
  });
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
