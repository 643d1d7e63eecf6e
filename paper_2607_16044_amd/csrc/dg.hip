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
// 1. face traces: T[e][f][q][0..3] = U, and for viscous flows [4..7] = F^nu(U, grad U) . n_e
//    (on far-field faces F^nu(U_inf, grad U) . n_e); records of 8 doubles, 4 when inviscid
//    A workgroup stages a tile of TE consecutive elements (their U, and Q of HDG-MX
//    elements) in LDS with coalesced loads; one thread per face point, and consecutive
//    threads write consecutive 64-byte point records.
// ---------------------------------------------------------------------------
template <int K> struct TraceTile {
  static constexpr int NQ = (3 * K + 2) / 2;
  static constexpr int TE = 256 / (4 * NQ);       // elements per workgroup: about 256 face points
};

template <int K, bool VISC>
__global__ void __launch_bounds__(256) dg_trace_kernel(DeviceMesh m, Gas g, int mx, const double* __restrict__ U,
                                                       const double* __restrict__ Q, double* __restrict__ T) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, TE = TraceTile<K>::TE;
  constexpr int NEV = VISC ? 2 : 1;                 // end values, and end derivatives for gradients
  constexpr int RS = VISC ? 8 : 4;                  // doubles per point record
  __shared__ double sU[TE * 4 * NN];
  __shared__ double sOut[TE * 4 * NQ * RS];         // records, staged for coalesced stores
  __shared__ double sQ[VISC ? TE * 5 * NN : 1];
  __shared__ double sE[TE][4][NEV][4][NP];          // U and dU across face f at its end, per line m
  __shared__ double sEQ[VISC ? TE : 1][4][5][NP];   // mixed variables at the face end (HDG-MX)
  __shared__ BasisTable tb;
  const int tid = threadIdx.x;
  const int base = blockIdx.x * TE;
  const int ne = min(TE, m.E - base);
  for (int i = tid; i < (int)(sizeof(BasisTable) / sizeof(double)); i += blockDim.x)
    reinterpret_cast<double*>(&tb)[i] = reinterpret_cast<const double*>(m.tab)[i];
  for (int i = tid; i < ne * 4 * NN; i += blockDim.x) sU[i] = U[(size_t)base * 4 * NN + i];
  if (VISC && mx)
    for (int i = tid; i < ne * 5 * NN; i += blockDim.x) {
      const int e = base + i / (5 * NN);
      sQ[i] = m.imp[e] ? Q[(size_t)base * 5 * NN + i] : 0.0;
    }
  __syncthreads();
  // phase 1: contraction across each face to its end (x-faces: over a at fixed b = m;
  // y-faces: over b at fixed a = m)
  for (int i = tid; i < ne * 4 * 4 * NP; i += blockDim.x) {
    const int mm = i % NP, v = (i / NP) % 4, f = (i / (4 * NP)) % 4, el = i / (16 * NP);
    const int s = f & 1;
    const double* u = sU + el * 4 * NN + v * NN;
    double e0 = 0.0, e1 = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const double x = (f < 2) ? u[j + NP * mm] : u[mm + NP * j];
      e0 += tb.LE[s][j] * x;
      if (VISC) e1 += tb.DE[s][j] * x;
    }
    sE[el][f][0][v][mm] = e0;
    if (VISC) sE[el][f][NEV - 1][v][mm] = e1;
  }
  if (VISC && mx)
    for (int i = tid; i < ne * 4 * 5 * NP; i += blockDim.x) {
      const int mm = i % NP, c = (i / NP) % 5, f = (i / (5 * NP)) % 4, el = i / (20 * NP);
      if (!m.imp[base + el]) continue;
      const int s = f & 1;
      const double* u = sQ + el * 5 * NN + c * NN;
      double e0 = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) e0 += tb.LE[s][j] * ((f < 2) ? u[j + NP * mm] : u[mm + NP * j]);
      sEQ[el][f][c][mm] = e0;
    }
  __syncthreads();
  // phase 2: one thread per face point, along the face
  if (tid < ne * 4 * NQ) {
  const int q = tid % NQ;
  const int f = (tid / NQ) % 4;
  const int el = tid / (4 * NQ);
  const int e = base + el;
  double val[4], dn[4], dt[4];                      // value, derivative across and along the face
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int mm = 0; mm < NP; ++mm) {
      const double e0 = sE[el][f][0][v][mm];
      a0 += tb.L[q][mm] * e0;
      if (VISC) {
        a1 += tb.L[q][mm] * sE[el][f][NEV - 1][v][mm];
        a2 += tb.D[q][mm] * e0;
      }
    }
    val[v] = a0;
    dn[v] = a1;
    dt[v] = a2;
  }
  double out[8];
#pragma unroll
  for (int v = 0; v < 4; ++v) { out[v] = val[v]; out[4 + v] = 0.0; }
  if (VISC) {
    double nx, ny;
    face_normal(f, nx, ny);
    if (mx && m.imp[e]) {
      double qv[5], F[4][2];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        double a0 = 0.0;
#pragma unroll
        for (int mm = 0; mm < NP; ++mm) a0 += tb.L[q][mm] * sEQ[el][f][c][mm];
        qv[c] = a0;
      }
      visc_flux_mx(val, qv, qv + 3, g, F);
#pragma unroll
      for (int v = 0; v < 4; ++v) out[4 + v] = F[v][0] * nx + F[v][1] * ny;
    } else {
      const double sx = 2.0 / m.hx[e], sy = 2.0 / m.hy[e];
      double G[4][2];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        G[v][0] = ((f < 2) ? dn[v] : dt[v]) * sx;
        G[v][1] = ((f < 2) ? dt[v] : dn[v]) * sy;
      }
      // boundary faces carry the far-field consistency flux K(U_inf) grad U . n
      const int far = m.nbr[e * 4 + f] < 0 && m.bcf[e * 4 + f] == IMEX_BC_FARFIELD;
      dg_face_visc_n(far, val, G, nx, ny, g, out + 4);
    }
  }
#pragma unroll
  for (int v = 0; v < RS; ++v) sOut[tid * RS + v] = out[v];
  }
  __syncthreads();
  // the tile's records are contiguous in T: consecutive threads store consecutive doubles
  double* o = T + (size_t)base * 4 * NQ * RS;
  for (int i = tid; i < ne * 4 * NQ * RS; i += blockDim.x) o[i] = sOut[i];
}

// ---------------------------------------------------------------------------
// 2. residual on a tile of ET explicit elements, sum-factorised
//    (eq. bilinear_form_interior_sdg tested with phi_n = l_a(xi) l_b(eta)):
//    P1  x-interpolation:  T0[v][b][i] = sum_a l_a(z_i) u[v][a,b],  T1 with l_a'
//    P2  volume points (i, j): u, du/dxi, du/deta from T0, T1 along y; fluxes F^nu - F^c
//        weighted by the rule; face points: traces, the neighbour's record, the face
//        integrand (numerical flux, consistency, penalty; adjoint coefficient)
//    P3  y-contraction of the volume coefficients, A[v][b][i] = sum_j l_b(z_j) Fx[j,i],
//        B[v][b][i] = sum_j l_b'(z_j) Fy[j,i], and the face line sums (each face's
//        points contracted with the 1D basis along the face)
//    P4  x-contraction: r[v][a,b] = sum_i (l_a'(z_i) A[b][i] + l_a(z_i) B[b][i]) plus the
//        face line sums times the end values l(+-1), l'(+-1) across the face
// ---------------------------------------------------------------------------
struct DGParams {
  int lf;            // Lax-Friedrichs instead of Vijayasundaram
  double alpha;      // IP penalty factor
};

template <int K> struct DGTile {
  static constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  // LDS doubles per element: U; x-interpolants (reused for the y-contraction); weighted
  // volume fluxes (x, y); face coefficients (s, d/dxi, d/deta); face line sums (2 per face)
  static constexpr int PER_EL = 4 * NN + 2 * 4 * NP * NQ + 2 * 4 * NQV + 4 * 3 * 4 * NQ + 4 * 2 * 4 * NP;
  static constexpr size_t lds(int et) { return 8 * ((size_t)et * PER_EL + sizeof(BasisTable) / 8) + 256; }
  // default: the largest power of two up to 32 whose tile stays within 48 KB
  static constexpr int ET = lds(32) <= 49152 ? 32 : lds(16) <= 49152 ? 16 : lds(8) <= 49152 ? 8
                            : lds(4) <= 49152 ? 4 : 2;
};
constexpr int DG_TILES[5] = {2, 4, 8, 16, 32};

// MODEL: DGM_GENERAL (runtime gas and flux flags) or DGM_EULER_LF (inviscid, Lax-Friedrichs,
// no far-field faces: the vortex workloads), which compiles only what that case needs
enum DGModel { DGM_GENERAL = 0, DGM_EULER_LF = 1 };

template <int K, int ET, int MODEL>
__global__ void __launch_bounds__(256) dg_residual_kernel(DeviceMesh m, Gas g, DGParams prm,
                                                          const int* __restrict__ ex_list, int n_ex,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ T, double* __restrict__ R) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  __shared__ double sU[ET][4][NN];
  __shared__ double sT[ET][2][4][NP][NQ];       // P1: x-interpolants; P3: y-contractions A, B
  __shared__ double sF[ET][2][4][NQV];          // weighted volume fluxes, x and y components
  __shared__ double sS[ET][4][3][4][NQ];        // face coefficients of phi, dphi/dxi, dphi/deta
  __shared__ double sL[ET][4][2][4][NP];        // face line sums
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
    (&sU[el][0][0])[r] = (e >= 0) ? U[(size_t)e * 4 * NN + r] : 0.0;
  }
  __syncthreads();
  // P1: interpolation along x at the Gauss abscissae
  for (int i = tid; i < ET * 4 * NP * NQ; i += blockDim.x) {
    const int qi = i % NQ, b = (i / NQ) % NP, v = (i / (NQ * NP)) % 4, el = i / (NQ * NP * 4);
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const double x = sU[el][v][a + NP * b];
      t0 += tb.L[qi][a] * x;
      t1 += tb.D[qi][a] * x;
    }
    sT[el][0][v][b][qi] = t0;
    sT[el][1][v][b][qi] = t1;
  }
  __syncthreads();
  // P2: volume points, then face points
  for (int i = tid; i < ET * (NQV + 4 * NQ); i += blockDim.x) {
    if (i < ET * NQV) {
      const int el = i / NQV, qv = i % NQV;
      const int e = sE[el];
      if (e < 0) continue;
      const int qi = qv % NQ, qj = qv / NQ;
      double val[4] = {0, 0, 0, 0}, dx[4] = {0, 0, 0, 0}, dy[4] = {0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        const double lb = tb.L[qj][b], db = tb.D[qj][b];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double t0 = sT[el][0][v][b][qi];
          val[v] += lb * t0;
          dy[v] += db * t0;
          dx[v] += lb * sT[el][1][v][b][qi];
        }
      }
      const double hx = m.hx[e], hy = m.hy[e];
      double Fc[4][2];
      conv_flux(val, g, Fc);
      double F[4][2];
#pragma unroll
      for (int v = 0; v < 4; ++v) { F[v][0] = -Fc[v][0]; F[v][1] = -Fc[v][1]; }
      if (MODEL == DGM_GENERAL && g.viscous) {
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
        sF[el][0][v][qv] = w * F[v][0] * (0.5 * hy);
        sF[el][1][v][qv] = w * F[v][1] * (0.5 * hx);
      }
    } else {
      const int k = i - ET * NQV;
      const int el = k / (4 * NQ), f = (k / NQ) % 4, q = k % NQ;
      const int e = sE[el];
      if (e < 0) continue;
      const double hx = m.hx[e], hy = m.hy[e];
      const double sx = 2.0 / hx, sy = 2.0 / hy;
      double nx, ny;
      face_normal(f, nx, ny);
      // own trace and consistency flux from this element's record (written by dg_trace)
      const int rs = (MODEL == DGM_GENERAL && g.viscous) ? 8 : 4;
      double Uo[4], fo[4] = {0, 0, 0, 0};
      const double* to = T + (((size_t)e * 4 + f) * NQ + q) * rs;
#pragma unroll
      for (int v = 0; v < 4; ++v) Uo[v] = to[v];
      if (rs == 8) {
#pragma unroll
        for (int v = 0; v < 4; ++v) fo[v] = to[4 + v];
      }
      const int nb = m.nbr[e * 4 + f];
      const double le = hx * hy / (2.0 * (hx + hy));
      double UN[4] = {0, 0, 0, 0}, fnn[4] = {0, 0, 0, 0};
      int kind = DGF_FARFIELD;
      double ln = le;
      if (nb >= 0) {
        kind = m.imp[nb] ? DGF_INTERFACE : DGF_INTERIOR;
        const double* tn = T + (((size_t)nb * 4 + (f ^ 1)) * NQ + q) * rs;
#pragma unroll
        for (int v = 0; v < 4; ++v) UN[v] = tn[v];
        if (rs == 8) {
#pragma unroll
          for (int v = 0; v < 4; ++v) fnn[v] = -tn[4 + v];     // neighbour's F^nu . n_e
        }
        ln = m.hx[nb] * m.hy[nb] / (2.0 * (m.hx[nb] + m.hy[nb]));
      }
      const double tau = dg_tau(prm.alpha, K, kind, le, ln);
      double s[4], gc[4][2];
      dg_face_point_fo<MODEL == DGM_EULER_LF>(kind, Uo, fo, UN, fnn, nx, ny, tau, prm.lf, g, s, gc);
      const double w = tb.W[q] * ((f < 2) ? 0.5 * hy : 0.5 * hx);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sS[el][f][0][v][q] = w * s[v];
        if (MODEL != DGM_EULER_LF) {                 // inviscid: no test-gradient term
          sS[el][f][1][v][q] = w * gc[v][0] * sx;
          sS[el][f][2][v][q] = w * gc[v][1] * sy;
        }
      }
    }
  }
  __syncthreads();
  // P3: y-contraction of the volume coefficients (into sT) and the face line sums
  for (int i = tid; i < ET * 4 * NP * (NQ + 4); i += blockDim.x) {
    if (i < ET * 4 * NP * NQ) {
      const int qi = i % NQ, b = (i / NQ) % NP, v = (i / (NQ * NP)) % 4, el = i / (NQ * NP * 4);
      double A = 0.0, B = 0.0;
#pragma unroll
      for (int qj = 0; qj < NQ; ++qj) {
        A += tb.L[qj][b] * sF[el][0][v][qi + NQ * qj];
        B += tb.D[qj][b] * sF[el][1][v][qi + NQ * qj];
      }
      sT[el][0][v][b][qi] = A;
      sT[el][1][v][b][qi] = B;
    } else {
      // face f, variable v, line index m (b for x-faces, a for y-faces)
      const int k = i - ET * 4 * NP * NQ;
      const int mm = k % NP, v = (k / NP) % 4, f = (k / (NP * 4)) % 4, el = k / (NP * 16);
      double P = 0.0, Qs = 0.0;
      if (MODEL == DGM_EULER_LF) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) P += sS[el][f][0][v][q] * tb.L[q][mm];
      } else if (f < 2) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          P += sS[el][f][0][v][q] * tb.L[q][mm] + sS[el][f][2][v][q] * tb.D[q][mm];
          Qs += sS[el][f][1][v][q] * tb.L[q][mm];
        }
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          P += sS[el][f][0][v][q] * tb.L[q][mm] + sS[el][f][1][v][q] * tb.D[q][mm];
          Qs += sS[el][f][2][v][q] * tb.L[q][mm];
        }
      }
      sL[el][f][0][v][mm] = P;
      sL[el][f][1][v][mm] = Qs;
    }
  }
  __syncthreads();
  // P4: x-contraction and the face terms, one thread per (element, variable, node)
  for (int i = tid; i < ET * 4 * NN; i += blockDim.x) {
    const int n = i % NN, v = (i / NN) % 4, el = i / (4 * NN);
    const int e = sE[el];
    if (e < 0) continue;
    const int a = n % NP, b = n / NP;
    double r = 0.0;
#pragma unroll
    for (int qi = 0; qi < NQ; ++qi) r += tb.D[qi][a] * sT[el][0][v][b][qi] + tb.L[qi][a] * sT[el][1][v][b][qi];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      r += tb.LE[s][a] * sL[el][s][0][v][b] + tb.LE[s][b] * sL[el][2 + s][0][v][a];       // x-, y-faces
      if (MODEL != DGM_EULER_LF)
        r += tb.DE[s][a] * sL[el][s][1][v][b] + tb.DE[s][b] * sL[el][2 + s][1][v][a];
    }
    R[(size_t)e * 4 * NN + v * NN + n] = r;
  }
}

// ---------------------------------------------------------------------------
// <Rbar, dR^DG/dp> along a far-field direction u_inf + p du (reverse mode of the far-field
// parameter): u_inf enters R^DG only at far-field faces of explicit elements (App. B.1.1),
// so the derivative is the far-field face integrand differentiated exactly by a dual
// number seeded in u_inf, tested against the trace and gradient of Rbar.  Per-block
// partial sums in part[gridDim.x].
// ---------------------------------------------------------------------------
struct Dir4 { double v[4]; };

template <int K>
__global__ void __launch_bounds__(256) dg_param_dot_kernel(DeviceMesh m, Gas g, double alpha,
                                                           const int* __restrict__ ex_list, int n_ex, Dir4 du,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ Rb, double* __restrict__ part) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP;
  using D1 = Dual<1>;
  __shared__ double red[4];
  const BasisTable& tb = *m.tab;
  double acc = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_ex * 4 * NQ; t += gridDim.x * blockDim.x) {
    const int q = t % NQ, f = (t / NQ) % 4, e = ex_list[t / (4 * NQ)];
    if (m.nbr[e * 4 + f] >= 0 || m.bcf[e * 4 + f] != IMEX_BC_FARFIELD) continue;
    const double hx = m.hx[e], hy = m.hy[e], sx = 2.0 / hx, sy = 2.0 / hy;
    double nx, ny;
    face_normal(f, nx, ny);
    double Uo[4], dxi[4], deta[4], rv[4], rx[4], ry[4];
    face_trace<K, 4>(tb, f, q, U + (size_t)e * 4 * NN, Uo, dxi, deta);
    face_trace<K, 4>(tb, f, q, Rb + (size_t)e * 4 * NN, rv, rx, ry);
    D1 Ui[4], fo[4], sd[4], gd[4][2];
    double Go[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ui[v] = D1(g.uinf[v]);
      Ui[v].d[0] = du.v[v];
      Go[v][0] = dxi[v] * sx;
      Go[v][1] = deta[v] * sy;
      fo[v] = D1(0.0);
    }
    if (g.viscous) {
      D1 Fv[4][2];
      visc_flux(Ui, Go, g, Fv);
#pragma unroll
      for (int v = 0; v < 4; ++v) fo[v] = Fv[v][0] * nx + Fv[v][1] * ny;
    }
    const double le = hx * hy / (2.0 * (hx + hy));
    dg_farfield_terms(Uo, fo, Ui, nx, ny, dg_tau(alpha, K, DGF_FARFIELD, le, le), g, sd, gd);
    const double w = tb.W[q] * ((f < 2) ? 0.5 * hy : 0.5 * hx);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      acc += w * (sd[v].d[0] * rv[v] + gd[v][0].d[0] * rx[v] * sx + gd[v][1].d[0] * ry[v] * sy);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// Manufactured-solution source (Sec. 5.1.1): U_e = (s, s, s, s^2), s = sin(a) + 4 with
// a = pi (kx x + ky y) - omega pi t.  U_e depends on (x, y) only through a, so
// div F(U_e, grad U_e) = pi (kx F_x + ky F_y)'(a): one dual number in a gives it, with
// grad U_e = pi k (x) dU_e/da carrying d2U_e/da2 as its derivative.
//   S = dU_e/dt + div(F^c - F^nu) = -omega pi dU_e/da + pi (kx (F^c - F^nu)_x + ky (...)_y)'
// b[e][v][n] = sum over volume points of w |J| S_v phi_n; one workgroup per element.
// ---------------------------------------------------------------------------
struct MMSParams { double kx, ky, omega, t; };

template <int K>
__global__ void __launch_bounds__(64) mms_load_kernel(DeviceMesh m, Gas g, MMSParams p,
                                                      const double* __restrict__ xy0, double* __restrict__ b) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  using D1 = Dual<1>;
  __shared__ double sS[NQV][4];
  const int e = blockIdx.x;
  const BasisTable& tb = *m.tab;
  const double hx = m.hx[e], hy = m.hy[e], jac = 0.25 * hx * hy;
  const double pi = 3.14159265358979323846;
  for (int qv = threadIdx.x; qv < NQV; qv += blockDim.x) {
    const int qi = qv % NQ, qj = qv / NQ;
    const double zi = tb.Z[qi], zj = tb.Z[qj];
    const double x = xy0[2 * e] + 0.5 * (zi + 1.0) * hx, y = xy0[2 * e + 1] + 0.5 * (zj + 1.0) * hy;
    const double arg = pi * (p.kx * x + p.ky * y) - p.omega * pi * p.t;
    const double sn = sin(arg), cs = cos(arg), s = sn + 4.0;
    const double dU[4] = {cs, cs, cs, 2.0 * s * cs};
    const double ddU[4] = {-sn, -sn, -sn, 2.0 * cs * cs - 2.0 * s * sn};
    const double Uv[4] = {s, s, s, s * s};
    D1 U[4], G[4][2], Fc[4][2], Fv[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      U[v] = D1(Uv[v]);
      U[v].d[0] = dU[v];
      G[v][0] = D1(pi * p.kx * dU[v]);
      G[v][0].d[0] = pi * p.kx * ddU[v];
      G[v][1] = D1(pi * p.ky * dU[v]);
      G[v][1].d[0] = pi * p.ky * ddU[v];
    }
    conv_flux(U, g, Fc);
    if (g.viscous) visc_flux(U, G, g, Fv);
    const double w = tb.W[qi] * tb.W[qj] * jac;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      D1 phi = p.kx * Fc[v][0] + p.ky * Fc[v][1];
      if (g.viscous) phi = phi - (p.kx * Fv[v][0] + p.ky * Fv[v][1]);
      sS[qv][v] = w * (-p.omega * pi * dU[v] + pi * phi.d[0]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * NN; i += blockDim.x) {
    const int v = i / NN, n = i % NN, a = n % NP, bb = n / NP;
    double acc = 0.0;
    for (int qj = 0; qj < NQ; ++qj)
      for (int qi = 0; qi < NQ; ++qi) acc += sS[qi + NQ * qj][v] * tb.L[qi][a] * tb.L[qj][bb];
    b[(size_t)e * 4 * NN + i] = acc;
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
  const int mx = (c->opt.hdg_variant == IMEX_HDG_MX) && c->gas.viscous && Q != nullptr;
  IMEX_DISPATCH_K(c->K, {
    constexpr int TE = TraceTile<KK>::TE;
    if (c->gas.viscous)
      hipLaunchKernelGGL((dg_trace_kernel<KK, true>), dim3((c->E + TE - 1) / TE), dim3(256), 0, c->stream,
                         c->dmesh(), c->gas, mx, U, Q, trace);
    else
      hipLaunchKernelGGL((dg_trace_kernel<KK, false>), dim3((c->E + TE - 1) / TE), dim3(256), 0, c->stream,
                         c->dmesh(), c->gas, mx, U, Q, trace);
  });
  return hipGetLastError();
}

template <int KK, int ET>
static bool launch_dg_tile(const imex_ctx* c, DGParams prm, const double* U, const double* trace, double* R) {
  if constexpr (DGTile<KK>::lds(ET) <= 65536) {
    const int nb = (c->n_ex + ET - 1) / ET;
    if (!c->gas.viscous && prm.lf && !c->dg_farfield)
      hipLaunchKernelGGL((dg_residual_kernel<KK, ET, DGM_EULER_LF>), dim3(nb), dim3(256), 0, c->stream, c->dmesh(),
                         c->gas, prm, c->d_ex_list, c->n_ex, U, trace, R);
    else
      hipLaunchKernelGGL((dg_residual_kernel<KK, ET, DGM_GENERAL>), dim3(nb), dim3(256), 0, c->stream, c->dmesh(),
                         c->gas, prm, c->d_ex_list, c->n_ex, U, trace, R);
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

hipError_t launch_dg_param_dot(const imex_ctx* c, const double* du, const double* U, const double* Rb, double* part,
                               int nblk) {
  Dir4 d{{du[0], du[1], du[2], du[3]}};
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(dg_param_dot_kernel<KK>, dim3(nblk), dim3(256), 0, c->stream, c->dmesh(),
                                           c->gas, c->opt.alpha_dg, c->d_ex_list, c->n_ex, d, U, Rb, part));
  return hipGetLastError();
}

hipError_t launch_mms_load(const imex_ctx* c, double t, double* b) {
  MMSParams p{c->mms[0], c->mms[1], c->mms[2], t};
  IMEX_DISPATCH_K(c->K, hipLaunchKernelGGL(mms_load_kernel<KK>, dim3(c->E), dim3(64), 0, c->stream, c->dmesh(),
                                           c->gas, p, c->d_xy0, b));
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
