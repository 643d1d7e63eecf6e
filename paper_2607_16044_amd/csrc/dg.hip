// Explicit DG-IP residual (Sec. 3.3), ERK stage combination (Sec. 4.2.2) and
// conservation sums on gfx950.
//
// R^DG is the weak-form operator of eq. bilinear_form_interior_sdg tested with
// each nodal basis function, with M dU/dt = -R.  Two launches per evaluation:
//  1. dg_trace: every element writes, at the Gauss points of its four faces,
//     its trace U and the normal viscous flux F^nu . n (outward normal of that
//     element); HDG-MX implicit elements use F^nu(U, eps, phi).  The buffer is
//     read by the neighbours, so every face flux is evaluated from data that was
//     computed once (no atomics, no neighbour gradients recomputed).
//  2. dg_residual: a workgroup owns a tile of explicit elements staged in LDS;
//     threads evaluate the volume fluxes at the volume Gauss points and the
//     numerical / interior-penalty face fluxes at the face points, then each
//     thread contracts them with the test functions of one node.
#include <mutex>

#include "ctx.h"
#include "dg_face.h"

namespace imex {

// ---------------------------------------------------------------------------
// Static device scratch of imex_dg_residual_noalloc (face traces and lifted mixed
// variables), for callers that cannot allocate.  One copy per device, resolved to a
// device address once per device with hipGetSymbolAddress; host code uses only that
// address, never the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;      // the device must be current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* static_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

__global__ void fill_zero_kernel(size_t n, double* __restrict__ x) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

hipError_t launch_fill_zero(const imex_ctx* c, double* x, size_t n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, x);
  return hipGetLastError();
}

// Trace of a nodal field (nv components, stride NN) and of its reference
// derivatives at Gauss point q of local face f.
template <int K, int NV>
__device__ inline void face_trace(const BasisTable& T, int f, int q, const double* u, double val[NV],
                                  double dxi[NV], double deta[NV]) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int s = f & 1;
#pragma unroll
  for (int v = 0; v < NV; ++v) { val[v] = 0.0; dxi[v] = 0.0; deta[v] = 0.0; }
  if (f < 2) {
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const double lb = T.L[q][b], db = T.D[q][b];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          const double x = u[v * NN + a + NP * b];
          t0 += T.LE[s][a] * x;
          t1 += T.DE[s][a] * x;
        }
        val[v] += lb * t0;
        dxi[v] += lb * t1;
        deta[v] += db * t0;
      }
    }
  } else {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const double la = T.L[q][a], da = T.D[q][a];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          const double x = u[v * NN + a + NP * b];
          t0 += T.LE[s][b] * x;
          t1 += T.DE[s][b] * x;
        }
        val[v] += la * t0;
        dxi[v] += da * t0;
        deta[v] += la * t1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 1. face traces: T[e][f][q][0..3] = U, [4..7] = F^nu(U, grad U) . n_e
// ---------------------------------------------------------------------------
template <int K>
__global__ void __launch_bounds__(256) dg_trace_kernel(DeviceMesh m, Gas g, int mx, const double* __restrict__ U,
                                                       const double* __restrict__ Q, double* __restrict__ T) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * 4 * NQ) return;
  const int q = t % NQ;
  const int f = (t / NQ) % 4;
  const int e = t / (4 * NQ);
  const BasisTable& tb = *m.tab;
  double val[4], dxi[4], deta[4];
  face_trace<K, 4>(tb, f, q, U + (size_t)e * 4 * NN, val, dxi, deta);
  double* out = T + (size_t)t * 8;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = val[v];
  if (!g.viscous) return;
  double nx, ny;
  face_normal(f, nx, ny);
  double F[4][2];
  if (mx && m.imp[e]) {
    double qv[5], qx[5], qy[5];
    face_trace<K, 5>(tb, f, q, Q + (size_t)e * 5 * NN, qv, qx, qy);
    visc_flux_mx(val, qv, qv + 3, g, F);
  } else {
    const double sx = 2.0 / m.hx[e], sy = 2.0 / m.hy[e];
    double G[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) { G[v][0] = dxi[v] * sx; G[v][1] = deta[v] * sy; }
    visc_flux(val, G, g, F);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) out[4 + v] = F[v][0] * nx + F[v][1] * ny;
}

// ---------------------------------------------------------------------------
// 2. residual on a tile of ET explicit elements
// ---------------------------------------------------------------------------
struct DGParams {
  int lf;            // Lax-Friedrichs instead of Vijayasundaram
  double alpha;      // IP penalty factor
};

// Elements per workgroup: the default fills about 256 volume points; other tiles
// are offered to the autotuner (imex_autotune) when their LDS fits in 64 KB.
template <int K> struct DGTile {
  static constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  static constexpr int ET0 = (256 / NQV) > 0 ? (256 / NQV) : 1;
  static constexpr int ET = ET0 > 32 ? 32 : ET0;
  static constexpr size_t lds(int et) { return 8 * (size_t)et * (4 * NN + NQV * 8 + 4 * NQ * 12) + 2048; }
};
constexpr int DG_TILES[5] = {2, 4, 8, 16, 32};

template <int K, int ET>
__global__ void __launch_bounds__(256) dg_residual_kernel(DeviceMesh m, Gas g, DGParams prm,
                                                          const int* __restrict__ ex_list, int n_ex,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ T, double* __restrict__ R) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  __shared__ double sU[ET][4 * NN];
  __shared__ double sF[ET][NQV][8];        // volume coefficients of d/dxi phi (0..3) and d/deta phi (4..7)
  __shared__ double sS[ET][4][NQ][4];      // face coefficients of phi
  __shared__ double sG[ET][4][NQ][8];      // face coefficients of d/dxi phi, d/deta phi
  __shared__ BasisTable tb;
  __shared__ int sE[ET];
  const int tid = threadIdx.x;
  const int base = blockIdx.x * ET;
  if (tid < ET) sE[tid] = (base + tid < n_ex) ? ex_list[base + tid] : -1;
  for (int i = tid; i < (int)(sizeof(BasisTable) / sizeof(double)); i += blockDim.x)
    reinterpret_cast<double*>(&tb)[i] = reinterpret_cast<const double*>(m.tab)[i];
  __syncthreads();
  for (int i = tid; i < ET * 4 * NN; i += blockDim.x) {
    const int el = i / (4 * NN), r = i % (4 * NN);
    const int e = sE[el];
    sU[el][r] = (e >= 0) ? U[(size_t)e * 4 * NN + r] : 0.0;
  }
  __syncthreads();
  // volume points
  for (int i = tid; i < ET * NQV; i += blockDim.x) {
    const int el = i / NQV, qv = i % NQV;
    const int e = sE[el];
    if (e < 0) continue;
    const int qi = qv % NQ, qj = qv / NQ;
    double val[4] = {0, 0, 0, 0}, dx[4] = {0, 0, 0, 0}, dy[4] = {0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const double lb = tb.L[qj][b], db = tb.D[qj][b];
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        const double la = tb.L[qi][a], da = tb.D[qi][a];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = sU[el][v * NN + a + NP * b];
          val[v] += la * lb * x;
          dx[v] += da * lb * x;
          dy[v] += la * db * x;
        }
      }
    }
    const double hx = m.hx[e], hy = m.hy[e];
    double Fc[4][2];
    conv_flux(val, g, Fc);
    double F[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) { F[v][0] = -Fc[v][0]; F[v][1] = -Fc[v][1]; }
    if (g.viscous) {
      double G[4][2], Fv[4][2];
#pragma unroll
      for (int v = 0; v < 4; ++v) { G[v][0] = dx[v] * (2.0 / hx); G[v][1] = dy[v] * (2.0 / hy); }
      visc_flux(val, G, g, Fv);
#pragma unroll
      for (int v = 0; v < 4; ++v) { F[v][0] += Fv[v][0]; F[v][1] += Fv[v][1]; }
    }
    // int F_x dphi/dx + F_y dphi/dy = sum_q w |J| (F_x (2/hx) dxi + F_y (2/hy) deta)
    const double w = tb.W[qi] * tb.W[qj];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sF[el][qv][v] = w * F[v][0] * (0.5 * hy);
      sF[el][qv][4 + v] = w * F[v][1] * (0.5 * hx);
    }
  }
  // face points
  for (int i = tid; i < ET * 4 * NQ; i += blockDim.x) {
    const int el = i / (4 * NQ), f = (i / NQ) % 4, q = i % NQ;
    const int e = sE[el];
    if (e < 0) continue;
    const double hx = m.hx[e], hy = m.hy[e];
    const double sx = 2.0 / hx, sy = 2.0 / hy;
    double nx, ny;
    face_normal(f, nx, ny);
    double Uo[4], dxi[4], deta[4];
    face_trace<K, 4>(tb, f, q, sU[el], Uo, dxi, deta);
    const int nb = m.nbr[e * 4 + f];
    const double le = hx * hy / (2.0 * (hx + hy));
    double G[4][2], UN[4] = {0, 0, 0, 0}, fnn[4] = {0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) { G[v][0] = dxi[v] * sx; G[v][1] = deta[v] * sy; }
    int kind = DGF_FARFIELD;
    double ln = le;
    if (nb >= 0) {
      kind = m.imp[nb] ? DGF_INTERFACE : DGF_INTERIOR;
      const double* tn = T + (((size_t)nb * 4 + (f ^ 1)) * NQ + q) * 8;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        UN[v] = tn[v];
        fnn[v] = -tn[4 + v];                 // neighbour's F^nu . n_e
      }
      ln = m.hx[nb] * m.hy[nb] / (2.0 * (m.hx[nb] + m.hy[nb]));
    }
    const double tau = dg_tau(prm.alpha, K, kind, le, ln);
    double s[4], gc[4][2];
    dg_face_point(kind, Uo, G, UN, fnn, nx, ny, tau, prm.lf, g, s, gc);
    const double w = tb.W[q] * ((f < 2) ? 0.5 * hy : 0.5 * hx);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sS[el][f][q][v] = w * s[v];
      sG[el][f][q][v] = w * gc[v][0] * sx;
      sG[el][f][q][4 + v] = w * gc[v][1] * sy;
    }
  }
  __syncthreads();
  // contraction with the test functions of node n = a + NP b
  for (int i = tid; i < ET * NN; i += blockDim.x) {
    const int el = i / NN, n = i % NN;
    const int e = sE[el];
    if (e < 0) continue;
    const int a = n % NP, b = n / NP;
    double r[4] = {0, 0, 0, 0};
    for (int qj = 0; qj < NQ; ++qj) {
#pragma unroll
      for (int qi = 0; qi < NQ; ++qi) {
        const int qv = qi + NQ * qj;
        const double px = tb.D[qi][a] * tb.L[qj][b];
        const double py = tb.L[qi][a] * tb.D[qj][b];
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] += sF[el][qv][v] * px + sF[el][qv][4 + v] * py;
      }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int s = f & 1;
      for (int q = 0; q < NQ; ++q) {
        double ph, pxi, peta;
        if (f < 2) {
          ph = tb.LE[s][a] * tb.L[q][b];
          pxi = tb.DE[s][a] * tb.L[q][b];
          peta = tb.LE[s][a] * tb.D[q][b];
        } else {
          ph = tb.L[q][a] * tb.LE[s][b];
          pxi = tb.D[q][a] * tb.LE[s][b];
          peta = tb.L[q][a] * tb.DE[s][b];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
          r[v] += sS[el][f][q][v] * ph + sG[el][f][q][v] * pxi + sG[el][f][q][4 + v] * peta;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) R[(size_t)e * 4 * NN + v * NN + n] = r[v];
  }
}

// ---------------------------------------------------------------------------
// ERK combination y = U_n - dt M^-1 sum_j c_j R_j on explicit elements
// ---------------------------------------------------------------------------
struct Terms {
  const double* R[8];
  double c[8];
  int n;
};

template <int K>
__global__ void erk_combine_kernel(DeviceMesh m, const int* __restrict__ ex_list, int n_ex,
                                   const double* __restrict__ Un, Terms terms, double dt, double* __restrict__ Y) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_ex * 4 * NN) return;
  const int r = t % (4 * NN);
  const int e = ex_list[t / (4 * NN)];
  const int n = r % NN;
  const BasisTable& tb = *m.tab;
  const double mass = tb.NW[n % NP] * tb.NW[n / NP] * m.hx[e] * m.hy[e] * 0.25;
  const size_t idx = (size_t)e * 4 * NN + r;
  double acc = 0.0;
  for (int j = 0; j < terms.n; ++j) acc += terms.c[j] * terms.R[j][idx];
  Y[idx] = Un[idx] - dt * elem_dt(m, e) * acc / mass;
}

// per-block partial sums of int_T U_v over all elements
template <int K>
__global__ void __launch_bounds__(256) mass_sum_kernel(DeviceMesh m, const double* __restrict__ U,
                                                       double* __restrict__ partial) {
  constexpr int NP = K + 1, NN = NP * NP;
  __shared__ double red[4][256];
  const int tid = threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  const BasisTable& tb = *m.tab;
  for (int i = blockIdx.x * blockDim.x + tid; i < m.E * NN; i += gridDim.x * blockDim.x) {
    const int e = i / NN, n = i % NN;
    const double w = tb.NW[n % NP] * tb.NW[n / NP] * m.hx[e] * m.hy[e] * 0.25;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += w * U[(size_t)e * 4 * NN + v * NN + n];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[v][tid] = acc[v];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int v = 0; v < 4; ++v) red[v][tid] += red[v][tid + s];
    }
    __syncthreads();
  }
  if (tid < 4) partial[blockIdx.x * 4 + tid] = red[tid][0];
}

__global__ void scale_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, double a,
                                  const double* __restrict__ add, double b, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = a * src[i] + (add ? b * add[i] : 0.0);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define IMEX_DISPATCH_K(KV, ...)                     \
  switch (KV) {                                      \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_dg_trace(const imex_ctx* c, const double* U, const double* Q, double* trace) {
  const int n = c->E * 4 * c->NQ;
  const int mx = (c->opt.hdg_variant == IMEX_HDG_MX) && c->gas.viscous && Q != nullptr;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(dg_trace_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                           c->dmesh(), c->gas, mx, U, Q, trace));
  return hipGetLastError();
}

template <int KK, int ET>
static bool launch_dg_tile(const imex_ctx* c, DGParams prm, const double* U, const double* trace, double* R) {
  if constexpr (DGTile<KK>::lds(ET) <= 65536) {
    const int nb = (c->n_ex + ET - 1) / ET;
    hipLaunchKernelGGL((dg_residual_kernel<KK, ET>), dim3(nb), dim3(256), 0, c->stream, c->dmesh(), c->gas, prm,
                       c->d_ex_list, c->n_ex, U, trace, R);
    return true;
  }
  return false;
}

bool dg_tile_valid(int K, int et) {
  if (et != 2 && et != 4 && et != 8 && et != 16 && et != 32) return false;   // the instantiated tiles
  switch (K) {
    case 1: return DGTile<1>::lds(et) <= 65536;
    case 2: return DGTile<2>::lds(et) <= 65536;
    case 3: return DGTile<3>::lds(et) <= 65536;
    case 4: return DGTile<4>::lds(et) <= 65536;
  }
  return false;
}

hipError_t launch_dg_residual(const imex_ctx* c, const double* U, const double* trace, double* R) {
  if (c->n_ex == 0) return hipSuccess;
  DGParams prm{c->opt.dg_flux == IMEX_FLUX_LAX_FRIEDRICHS, c->opt.alpha_dg};
  IMEX_DISPATCH_K(c->K, {
    bool ok = true;
    switch (c->dg_tile) {
      case 2: ok = launch_dg_tile<KK, 2>(c, prm, U, trace, R); break;
      case 4: ok = launch_dg_tile<KK, 4>(c, prm, U, trace, R); break;
      case 8: ok = launch_dg_tile<KK, 8>(c, prm, U, trace, R); break;
      case 16: ok = launch_dg_tile<KK, 16>(c, prm, U, trace, R); break;
      case 32: ok = launch_dg_tile<KK, 32>(c, prm, U, trace, R); break;
      default: ok = launch_dg_tile<KK, DGTile<KK>::ET>(c, prm, U, trace, R); break;
    }
    if (!ok) return hipErrorInvalidValue;
  });
  return hipGetLastError();
}

hipError_t launch_erk_combine(const imex_ctx* c, const double* Un, int nterms, const double* const* R,
                              const double* coef, double dt, double* Y) {
  if (c->n_ex == 0) return hipSuccess;
  if (nterms > 8) return hipErrorInvalidValue;
  Terms t{};
  t.n = 0;
  for (int j = 0; j < nterms; ++j) {
    if (coef[j] == 0.0) continue;
    t.R[t.n] = R[j];
    t.c[t.n] = coef[j];
    ++t.n;
  }
  const int n = c->n_ex * 4 * c->NN;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(erk_combine_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                           c->dmesh(), c->d_ex_list, c->n_ex, Un, t, dt, Y));
  return hipGetLastError();
}

hipError_t launch_mass_sums(const imex_ctx* c, const double* U, double* partial, int* nblocks) {
  const int nb = 256;
  *nblocks = nb;
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(mass_sum_kernel<KK>, dim3(nb), dim3(256), 0, c->stream, c->dmesh(), U,
                                           partial));
  return hipGetLastError();
}

hipError_t launch_scale_copy(const imex_ctx* c, const double* src, double* dst, double a, const double* add,
                             double b, size_t n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, src, dst, a,
                     add, b, n);
  return hipGetLastError();
}

}  // namespace imex
