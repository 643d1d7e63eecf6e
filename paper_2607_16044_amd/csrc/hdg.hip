// Implicit HDG stage (Sec. 4.3): Newton with static condensation and a GMRES
// facet solve, on gfx950.
//
// Per Newton iteration:
//  1. hdg_assemble   one workgroup per implicit element: residual rows f, the
//                    element's facet rows h and the blocks K, C, D, E of the
//                    linearisation in (U_T, Uhat on dT) (eq. implicit_system).
//                    Point-wise flux Jacobians come from dual numbers and are
//                    contracted with the basis; HDG-MX mixed variables are lifted
//                    from (U, Uhat) and their blocks A12, A21, A23, A32 stored.
//  2. hdg_eliminate  (HDG-MX) removes the mixed block: A22 is the diagonal mass
//                    matrix, so K -= A12 A22^-1 A21 etc. exactly.
//  3. hdg_condense   in-LDS LU with partial pivoting of K; X = K^-1 C,
//                    y = K^-1 f, S_T = E - D X, r_T = D y (eqs.
//                    statically_condensed_system, SchurCompliment).
//  4. facet solve    right-preconditioned restarted GMRES on S dUhat = -h + sum r_T
//                    with per-facet block-Jacobi; S is applied facet by facet from
//                    the stored S_T blocks of the (at most two) adjacent elements.
//  5. hdg_backsub    dU_T = -y_T - X_T dUhat_T (eq. local_solve_static_condensation),
//                    update and increment norms.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ctx.h"

namespace imex {

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
template <int K, bool MX> struct HS {
  static constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  static constexpr int NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP;
  static constexpr int NQM = MX ? 5 * NN : 0;
  static constexpr int NIV = MX ? 9 : 12;     // volume point inputs: U + (Q | grad U)
  static constexpr int NIF = MX ? 13 : 16;    // face point inputs: U + Uhat + (Q | grad U)
  static constexpr int NOF = MX ? 8 : 16;     // face point outputs: s + t (+ g for IP)
  static constexpr int NR = NU + NF, NC = NU + NF + 1;       // augmented local system [[K C f],[D E h]]
  static constexpr size_t BLK = (size_t)NR * NC;
  static constexpr size_t SCR = MX ? 2 * (size_t)NR * NQM : 0;  // L = [A12; A32], R = M_Q^-1 [A21 A23]
};

__device__ __forceinline__ void fnormal(int f, double& nx, double& ny) {
  nx = (f == 0) ? -1.0 : (f == 1 ? 1.0 : 0.0);
  ny = (f == 2) ? -1.0 : (f == 3 ? 1.0 : 0.0);
}

// basis value and reference derivatives of node n = a + NP b at face point (f, q)
template <int K>
__device__ __forceinline__ void face_basis(const BasisTable& tb, int f, int q, int a, int b, double& ph,
                                           double& pxi, double& peta) {
  const int s = f & 1;
  if (f < 2) {
    ph = tb.LE[s][a] * tb.L[q][b];
    pxi = tb.DE[s][a] * tb.L[q][b];
    peta = tb.LE[s][a] * tb.D[q][b];
  } else {
    ph = tb.L[q][a] * tb.LE[s][b];
    pxi = tb.D[q][a] * tb.LE[s][b];
    peta = tb.L[q][a] * tb.DE[s][b];
  }
}

// ---------------------------------------------------------------------------
// point functions (templated on the scalar for value / dual evaluation)
// ---------------------------------------------------------------------------
struct FaceData {
  int kind;
  double nx, ny, tau;
  double uex[4];
  int lf;
};

// volume: out = F^nu - F^c ; IP/Euler uses grad U, MX the mixed variables
template <class T>
__device__ inline void vol_point_ip(const T W[4], const T G[4][2], const Gas& g, T out[4][2]) {
  conv_flux(W, g, out);
#pragma unroll
  for (int v = 0; v < 4; ++v) { out[v][0] = -out[v][0]; out[v][1] = -out[v][1]; }
  if (g.viscous) {
    T Fv[4][2];
    visc_flux(W, G, g, Fv);
#pragma unroll
    for (int v = 0; v < 4; ++v) { out[v][0] = out[v][0] + Fv[v][0]; out[v][1] = out[v][1] + Fv[v][1]; }
  }
}

template <class T>
__device__ inline void vol_point_mx(const T W[4], const T Q[5], const Gas& g, T out[4][2]) {
  conv_flux(W, g, out);
#pragma unroll
  for (int v = 0; v < 4; ++v) { out[v][0] = -out[v][0]; out[v][1] = -out[v][1]; }
  T Fv[4][2];
  visc_flux_mx(W, Q, Q + 3, g, Fv);
#pragma unroll
  for (int v = 0; v < 4; ++v) { out[v][0] = out[v][0] + Fv[v][0]; out[v][1] = out[v][1] + Fv[v][1]; }
}

// HDG-IP face point (eq. bilinear_form_interior_hdg_ip_element / _facet, App. B.2):
// s = coefficient of V, gc = coefficient of grad V, t = facet row integrand.
template <class T>
__device__ inline void face_point_ip(const T W[4], const T G[4][2], const T Wh[4], const FaceData& fd, const Gas& g,
                                     T s[4], T gc[4][2], T t[4]) {
  const double nx = fd.nx, ny = fd.ny;
  T Fc[4];
  hdg_num_flux(W, Wh, nx, ny, fd.lf, g, Fc);
#pragma unroll
  for (int v = 0; v < 4; ++v) { s[v] = Fc[v]; gc[v][0] = T(0.0); gc[v][1] = T(0.0); }
  T visc_n[4];     // F^nu_n(Uh, grad U) - tau K(Uh)(U - Uh) (x) n . n
#pragma unroll
  for (int v = 0; v < 4; ++v) visc_n[v] = T(0.0);
  if (g.viscous) {
    const int wall = fd.kind == FK_WALL;
    T Kg[4][2], Gj[4][2], Kj[4][2];
    visc_flux(Wh, G, g, Kg, wall, nx, ny);
#pragma unroll
    for (int v = 0; v < 4; ++v) { const T d = W[v] - Wh[v]; Gj[v][0] = d * nx; Gj[v][1] = d * ny; }
    visc_flux(Wh, Gj, g, Kj, wall, nx, ny);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T kgn = Kg[v][0] * nx + Kg[v][1] * ny;
      const T kjn = Kj[v][0] * nx + Kj[v][1] * ny;
      s[v] = s[v] - kgn + fd.tau * kjn;
      gc[v][0] = -Kj[v][0];
      gc[v][1] = -Kj[v][1];
      visc_n[v] = kgn - fd.tau * kjn;
    }
  }
  if (fd.kind == FK_INTERIOR) {
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = visc_n[v] - Fc[v];
  } else if (fd.kind == FK_INTERFACE) {
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = Wh[v] - fd.uex[v];
  } else if (fd.kind == FK_FARFIELD) {
    T d1[4], d2[4], a1[4], a2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) { d1[v] = Wh[v] - W[v]; d2[v] = Wh[v] - g.uinf[v]; }
    char_apply(Wh, d1, nx, ny, +1, g, a1);
    char_apply(Wh, d2, nx, ny, -1, g, a2);
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = a1[v] - a2[v];
  } else {   // adiabatic wall: Uhat = (rho, 0, 0, rho e_i) of the trace
    const T rei = W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0];
    t[0] = Wh[0] - W[0];
    t[1] = Wh[1];
    t[2] = Wh[2];
    t[3] = Wh[3] - rei;
  }
}

// HDG-MX face point (eq. bilinear_form_hdg_mixed, eq. viscous_numerical_flux, App. B.3)
template <class T>
__device__ inline void face_point_mx(const T W[4], const T Wh[4], const T Q[5], const FaceData& fd, const Gas& g,
                                     T s[4], T t[4]) {
  const double nx = fd.nx, ny = fd.ny;
  T Fc[4];
  hdg_num_flux(W, Wh, nx, ny, fd.lf, g, Fc);
  T Fv[4][2];
  visc_flux_mx(Wh, Q, Q + 3, g, Fv);
  const double Sd[4] = {0.0, g.mu, g.mu, g.kappa};
#pragma unroll
  for (int v = 0; v < 4; ++v) s[v] = Fc[v] - (Fv[v][0] * nx + Fv[v][1] * ny - Sd[v] * (W[v] - Wh[v]));
  if (fd.kind == FK_INTERIOR) {
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = s[v];
  } else if (fd.kind == FK_INTERFACE) {
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = Wh[v] - fd.uex[v];
  } else if (fd.kind == FK_FARFIELD) {
    T d1[4], d2[4], a1[4], a2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) { d1[v] = Wh[v] - W[v]; d2[v] = Wh[v] - g.uinf[v]; }
    char_apply(Wh, d1, nx, ny, +1, g, a1);
    char_apply(Wh, d2, nx, ny, -1, g, a2);
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = a1[v] - a2[v];
  } else {   // adiabatic wall (App. B.3.2)
    t[0] = Wh[0] - W[0];
    t[1] = Wh[1];
    t[2] = Wh[2];
    t[3] = g.kappa * (Q[3] * nx + Q[4] * ny) - g.kappa * (W[3] - Wh[3]);
  }
}

// primitive quantities entering the mixed lifting: (u, v, theta)
template <class T> __device__ inline void lift_point(const T W[4], const Gas& g, T P[3]) {
  const T ir = 1.0 / W[0];
  P[0] = W[1] * ir;
  P[1] = W[2] * ir;
  P[2] = (W[3] * ir - 0.5 * (P[0] * P[0] + P[1] * P[1])) * (1.0 / g.cv);
}

// ---------------------------------------------------------------------------
// assembly
// ---------------------------------------------------------------------------
// dual-number seeds per pass of the point-wise Jacobians (1, 2 or 4)
#ifndef ASM_SEEDS
#define ASM_SEEDS 1
#endif
static_assert(ASM_SEEDS == 1 || ASM_SEEDS == 2 || ASM_SEEDS == 4, "seeds per pass");
// optional bound on the assembly kernel's waves per SIMD (0: the compiler's choice)
#ifndef ASM_WAVES_PER_EU
#define ASM_WAVES_PER_EU 0
#endif
#if ASM_WAVES_PER_EU > 0
#define ASM_WAVES __attribute__((amdgpu_waves_per_eu(ASM_WAVES_PER_EU, ASM_WAVES_PER_EU)))
#else
#define ASM_WAVES
#endif

struct AsmParams {
  double dt_a;
  double alpha;
  int lf;
  int jacobian;      // 0: residual only
};

// DUMP: the point-wise Jacobians go straight to the element's record in global memory
// (same layout), so the workgroup's LDS holds only the values and several elements
// share a CU.
template <int K, bool MX, bool DUMP = false> struct AsmShared {
  using S = HS<K, MX>;
  static constexpr int NJV = DUMP ? 1 : S::NQV, NJF = DUMP ? 1 : 4, NJL = (MX && !DUMP) ? S::NQV : 1,
                       NJLF = (MX && !DUMP) ? 4 : 1;
  BasisTable tb;
  double U[S::NU];
  double Uh[S::NF];                   // [face][v][m]
  double Q[MX ? S::NQM : 1];          // [c][n]
  double uex[4][S::NQ][4];
  double VV[S::NQV][8];               // volume point outputs
  double JV[NJV][8][S::NIV];          // d out / d in at volume points
  double VF[4][S::NQ][S::NOF];        // face point outputs
  double JF[NJF][S::NQ][S::NOF][S::NIF];
  double PL[S::NQV][3];               // lifting inputs at volume points (MX)
  double JL[NJL][3][4];
  double PLF[4][S::NQ][3];
  double JLF[NJLF][S::NQ][3][4];
  double Gv[S::NQV][8];               // grad U at volume points (IP)
  double Gf[4][S::NQ][8];             // grad U at face points (IP)
  double Wv[S::NQV][4];
  double Wf[4][S::NQ][4];
  double Wh[4][S::NQ][4];
  double Qv[MX ? S::NQV : 1][5];
  double Qf[MX ? 4 : 1][S::NQ][5];
};

// Point-wise record of one element written by the assembly kernel in point mode
// and read by the block contraction: d(volume flux)/d(U, Q | grad U) at the
// volume points, d(face outputs)/d(U, Uhat, Q | grad U) at the face points and,
// for HDG-MX, the derivatives of the lifted primitives (u, v, theta) with
// respect to U (volume points) and Uhat (face points).  Face outputs: HDG-MX
// (s, t); HDG-IP (s, coefficient of grad V, t).
template <int K, bool MX> struct PointRec {
  static constexpr int NQ = (3 * K + 2) / 2, NQV = NQ * NQ;
  static constexpr int NIV = MX ? 9 : 12, NOF = MX ? 8 : 16, NIF = MX ? 13 : 16;
  static constexpr int TO = MX ? 4 : 12;              // t rows among the face outputs
  static constexpr int JV = 0;                        // [NQV][8][NIV]
  static constexpr int JF = JV + NQV * 8 * NIV;       // [4][NQ][NOF][NIF]
  static constexpr int JL = JF + 4 * NQ * NOF * NIF;  // [NQV][3][4]      (HDG-MX)
  static constexpr int JLF = JL + (MX ? NQV * 12 : 0);// [4][NQ][3][4]    (HDG-MX)
  static constexpr int SIZE = JLF + (MX ? 4 * NQ * 12 : 0);
};
template <int K> using MxRec = PointRec<K, true>;

// Residual rows here; the point-wise Jacobians go to rec, which hdg_contract_kernel
// (HDG-MX, inviscid HDG-IP) or hdg_contract_ipv_kernel (viscous HDG-IP) contracts into
// the element blocks.  (DUMP = true is the only mode: it selects the record as the
// destination of the point Jacobians.)
// JAC = false: point values and residual rows only (a separate instantiation without the
// dual-number passes).
// EPB elements per workgroup (256 / EPB threads each, one LDS slot each).  The kernel's
// register budget allows one wave per SIMD, so a workgroup is all that a CU runs: with
// one element per workgroup its waves would idle through the element's serial phases and
// short task lists (77 point tasks at k = 4 in the residual-only pass).  A slot past the
// last element repeats the last element (identical values to the same addresses).  Eight
// elements at k = 1 and for the k = 2 Jacobian pass; four otherwise (the k = 2 residual-only
// pass was slower with eight).
template <int K, bool MX, bool JAC> constexpr int asm_epb() {
  return (K == 1 || (JAC && K == 2)) ? 8 : 4;
}
template <int K, bool MX, bool DUMP> constexpr size_t asm_slot_doubles() {
  return (sizeof(AsmShared<K, MX, DUMP>) + 15) / 16 * 2;
}

template <int K, bool MX, bool DUMP, class T, bool JAC = true>
__global__ void __launch_bounds__(256) ASM_WAVES hdg_assemble_kernel(DeviceMesh m, DeviceHDG h, Gas g, AsmParams prm,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ Uhat,
                                                           const double* __restrict__ rhs, T* __restrict__ blk,
                                                           T* __restrict__ scr, double* __restrict__ Qout,
                                                           double* __restrict__ Rh, double* __restrict__ rec,
                                                           double* __restrict__ hres) {
  using S = HS<K, MX>;
  static_assert(DUMP, "the point Jacobians go to the record");
  constexpr int NP = S::NP, NQ = S::NQ, NN = S::NN, NQV = S::NQV, NU = S::NU, NF = S::NF, NFF = S::NFF;
  constexpr int NQM = S::NQM, NIV = S::NIV, NIF = S::NIF, NOF = S::NOF;
  constexpr int EPB = asm_epb<K, MX, JAC>(), TPE = 256 / EPB;
  static_assert(sizeof(double) * asm_slot_doubles<K, MX, DUMP || !JAC>() * EPB <= 160 * 1024, "LDS per workgroup");
  const int slot = threadIdx.x / TPE;
  const int p = min((int)blockIdx.x * EPB + slot, h.n_im - 1);
  extern __shared__ double smem_raw[];
  AsmShared<K, MX, DUMP || !JAC>& sh = *reinterpret_cast<AsmShared<K, MX, DUMP || !JAC>*>(
      smem_raw + (size_t)slot * asm_slot_doubles<K, MX, DUMP || !JAC>());
  using Rec = PointRec<K, MX>;
  double* const rp = DUMP ? rec + (size_t)p * Rec::SIZE : nullptr;
  // point-wise Jacobian entries: LDS, or the record in global memory (DUMP)
  auto jv = [&](int qv, int o, int col) -> double& {
    if constexpr (DUMP) return rp[Rec::JV + ((size_t)qv * 8 + o) * NIV + col];
    else return sh.JV[qv][o][col];
  };
  auto jf = [&](int f, int q, int o, int col) -> double& {
    if constexpr (DUMP) return rp[Rec::JF + (((size_t)f * NQ + q) * NOF + o) * NIF + col];
    else return sh.JF[f][q][o][col];
  };
  auto jl = [&](int qv, int c, int v) -> double& {
    if constexpr (DUMP) return rp[Rec::JL + ((size_t)qv * 3 + c) * 4 + v];
    else return sh.JL[MX ? qv : 0][c][v];
  };
  auto jlf = [&](int f, int q, int c, int v) -> double& {
    if constexpr (DUMP) return rp[Rec::JLF + (((size_t)f * NQ + q) * 3 + c) * 4 + v];
    else return sh.JLF[MX ? f : 0][q][c][v];
  };
  const int e = h.im_list[p];
  const int tid = threadIdx.x % TPE, nt = TPE;
  for (int i = tid; i < (int)(sizeof(BasisTable) / sizeof(double)); i += nt)
    reinterpret_cast<double*>(&sh.tb)[i] = reinterpret_cast<const double*>(m.tab)[i];
  for (int i = tid; i < NU; i += nt) sh.U[i] = U[(size_t)e * NU + i];
  for (int i = tid; i < NF; i += nt) {
    const int f = i / NFF, r = i % NFF;
    sh.Uh[i] = Uhat[(size_t)h.efacet[4 * p + f] * NFF + r];
  }
  __syncthreads();
  const BasisTable& tb = sh.tb;
  const double hx = m.hx[e], hy = m.hy[e];
  const double sx = 2.0 / hx, sy = 2.0 / hy, jac = 0.25 * hx * hy;
  const double dta = prm.dt_a * elem_dt(m, e);      // dt a_ii of this element's instance
  const double le = hx * hy / (2.0 * (hx + hy));
  const double tau = prm.alpha * (double)((K + 1) * (K + 1)) / le;
  // ---- point values -----------------------------------------------------
  for (int qv = tid; qv < NQV; qv += nt) {
    const int qi = qv % NQ, qj = qv / NQ;
    double W[4] = {0, 0, 0, 0}, gx[4] = {0, 0, 0, 0}, gy[4] = {0, 0, 0, 0};
    for (int b = 0; b < NP; ++b)
      for (int a = 0; a < NP; ++a) {
        const double ph = tb.L[qi][a] * tb.L[qj][b];
        const double px = tb.D[qi][a] * tb.L[qj][b] * sx;
        const double py = tb.L[qi][a] * tb.D[qj][b] * sy;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = sh.U[v * NN + a + NP * b];
          W[v] += ph * x;
          gx[v] += px * x;
          gy[v] += py * x;
        }
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sh.Wv[qv][v] = W[v];
      sh.Gv[qv][2 * v] = gx[v];
      sh.Gv[qv][2 * v + 1] = gy[v];
    }
    if (MX) {
      double P[3];
      lift_point(W, g, P);
      for (int c = 0; c < 3; ++c) sh.PL[qv][c] = P[c];
    }
  }
  for (int i = tid; i < 4 * NQ; i += nt) {
    const int f = i / NQ, q = i % NQ;
    double W[4] = {0, 0, 0, 0}, gx[4] = {0, 0, 0, 0}, gy[4] = {0, 0, 0, 0}, Wh[4] = {0, 0, 0, 0};
    for (int b = 0; b < NP; ++b)
      for (int a = 0; a < NP; ++a) {
        double ph, pxi, peta;
        face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = sh.U[v * NN + a + NP * b];
          W[v] += ph * x;
          gx[v] += pxi * sx * x;
          gy[v] += peta * sy * x;
        }
      }
    for (int mm = 0; mm < NP; ++mm) {
      const double ps = tb.L[q][mm];
#pragma unroll
      for (int v = 0; v < 4; ++v) Wh[v] += ps * sh.Uh[f * NFF + v * NP + mm];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sh.Wf[f][q][v] = W[v];
      sh.Gf[f][q][2 * v] = gx[v];
      sh.Gf[f][q][2 * v + 1] = gy[v];
      sh.Wh[f][q][v] = Wh[v];
    }
    if (MX) {
      double P[3];
      lift_point(Wh, g, P);
      for (int c = 0; c < 3; ++c) sh.PLF[f][q][c] = P[c];
    }
    // interface data: the explicit neighbour's trace
    double ux[4] = {0, 0, 0, 0};
    if (h.face_kind[4 * p + f] == FK_INTERFACE) {
      const int nb = m.nbr[4 * e + f];
      const int fo = f ^ 1;
      for (int b = 0; b < NP; ++b)
        for (int a = 0; a < NP; ++a) {
          double ph, pxi, peta;
          face_basis<K>(tb, fo, q, a, b, ph, pxi, peta);
#pragma unroll
          for (int v = 0; v < 4; ++v) ux[v] += ph * U[(size_t)nb * NU + v * NN + a + NP * b];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sh.uex[f][q][v] = ux[v];
  }
  __syncthreads();
  // ---- mixed variables Q = -M_Q^-1 l(U, Uhat) (HDG-MX) ----------------
  if (MX) {
    for (int n = tid; n < NN; n += nt) {
      const int a = n % NP, b = n / NP;
      double l[5] = {0, 0, 0, 0, 0};
      for (int qj = 0; qj < NQ; ++qj)
        for (int qi = 0; qi < NQ; ++qi) {
          const int qv = qi + NQ * qj;
          const double w = tb.W[qi] * tb.W[qj] * jac;
          const double px = w * tb.D[qi][a] * tb.L[qj][b] * sx;
          const double py = w * tb.L[qi][a] * tb.D[qj][b] * sy;
          const double u = sh.PL[qv][0], v = sh.PL[qv][1], th = sh.PL[qv][2];
          l[0] += (2.0 / 3.0) * u * px - (1.0 / 3.0) * v * py;
          l[1] += u * py + v * px;
          l[2] += -(1.0 / 3.0) * u * px + (2.0 / 3.0) * v * py;
          l[3] += th * px;
          l[4] += th * py;
        }
      for (int f = 0; f < 4; ++f) {
        double nx, ny;
        fnormal(f, nx, ny);
        const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
        for (int q = 0; q < NQ; ++q) {
          double ph, pxi, peta;
          face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
          ph *= tb.W[q] * wl;
          const double u = sh.PLF[f][q][0], v = sh.PLF[f][q][1], th = sh.PLF[f][q][2];
          l[0] -= ph * ((2.0 / 3.0) * u * nx - (1.0 / 3.0) * v * ny);
          l[1] -= ph * (u * ny + v * nx);
          l[2] -= ph * (-(1.0 / 3.0) * u * nx + (2.0 / 3.0) * v * ny);
          l[3] -= ph * th * nx;
          l[4] -= ph * th * ny;
        }
      }
      const double mass = tb.NW[a] * tb.NW[b] * jac;
      const double fac[5] = {1.0, 2.0, 1.0, 1.0, 1.0};
      for (int c = 0; c < 5; ++c) {
        const double qval = -l[c] / (fac[c] * mass);
        sh.Q[c * NN + n] = qval;
        if (Qout) Qout[(size_t)e * 5 * NN + c * NN + n] = qval;
      }
    }
    __syncthreads();
    for (int qv = tid; qv < NQV; qv += nt) {
      const int qi = qv % NQ, qj = qv / NQ;
      double qq[5] = {0, 0, 0, 0, 0};
      for (int b = 0; b < NP; ++b)
        for (int a = 0; a < NP; ++a) {
          const double ph = tb.L[qi][a] * tb.L[qj][b];
          for (int c = 0; c < 5; ++c) qq[c] += ph * sh.Q[c * NN + a + NP * b];
        }
      for (int c = 0; c < 5; ++c) sh.Qv[qv][c] = qq[c];
    }
    for (int i = tid; i < 4 * NQ; i += nt) {
      const int f = i / NQ, q = i % NQ;
      double qq[5] = {0, 0, 0, 0, 0};
      for (int b = 0; b < NP; ++b)
        for (int a = 0; a < NP; ++a) {
          double ph, pxi, peta;
          face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
          for (int c = 0; c < 5; ++c) qq[c] += ph * sh.Q[c * NN + a + NP * b];
        }
      for (int c = 0; c < 5; ++c) sh.Qf[f][q][c] = qq[c];
    }
    __syncthreads();
  }
  // ---- point-wise outputs and Jacobians (dual numbers, NSD seeds per pass) ----
  // Fewer seeds per pass cost more passes but far fewer registers per task.
  constexpr int NSD = ASM_SEEDS;
  constexpr int CV0 = (NIV + NSD - 1) / NSD, CF0 = (NIF + NSD - 1) / NSD, CL = 4 / NSD;
  // inviscid HDG-IP: the outputs do not depend on grad U, only the chunks of U (and Uhat)
  const bool full = MX || g.viscous || !DUMP;
  const int CV = full ? CV0 : 4 / NSD, CF = full ? CF0 : 8 / NSD;
  const int ntask = NQV * CV + 4 * NQ * CF + (MX ? (NQV + 4 * NQ) * CL : 0);
  for (int task = tid; task < (JAC ? ntask : NQV + 4 * NQ); task += nt) {
    if constexpr (!JAC) {
      // values only
      if (task < NQV) {
        const int qv = task;
        double out[4][2];
        if (MX) vol_point_mx(sh.Wv[qv], sh.Qv[qv], g, out);
        else {
          double G[4][2];
          for (int v = 0; v < 4; ++v) { G[v][0] = sh.Gv[qv][2 * v]; G[v][1] = sh.Gv[qv][2 * v + 1]; }
          vol_point_ip(sh.Wv[qv], G, g, out);
        }
        for (int v = 0; v < 4; ++v) { sh.VV[qv][2 * v] = out[v][0]; sh.VV[qv][2 * v + 1] = out[v][1]; }
      } else {
        const int i = task - NQV, f = i / NQ, q = i % NQ;
        FaceData fd;
        fd.kind = h.face_kind[4 * p + f];
        fnormal(f, fd.nx, fd.ny);
        fd.tau = tau;
        fd.lf = prm.lf;
        for (int v = 0; v < 4; ++v) fd.uex[v] = sh.uex[f][q][v];
        if (MX) {
          double s[4], t[4];
          face_point_mx(sh.Wf[f][q], sh.Wh[f][q], sh.Qf[f][q], fd, g, s, t);
          for (int v = 0; v < 4; ++v) { sh.VF[f][q][v] = s[v]; sh.VF[f][q][4 + v] = t[v]; }
        } else {
          double G[4][2], s[4], gc[4][2], t[4];
          for (int v = 0; v < 4; ++v) { G[v][0] = sh.Gf[f][q][2 * v]; G[v][1] = sh.Gf[f][q][2 * v + 1]; }
          face_point_ip(sh.Wf[f][q], G, sh.Wh[f][q], fd, g, s, gc, t);
          for (int v = 0; v < 4; ++v) {
            sh.VF[f][q][v] = s[v];
            sh.VF[f][q][4 + 2 * v] = gc[v][0];
            sh.VF[f][q][5 + 2 * v] = gc[v][1];
            sh.VF[f][q][12 + v] = t[v];
          }
        }
      }
      continue;
    }
    using D4 = Dual<NSD>;
    if (task < NQV * CV) {
      const int qv = task / CV, ch = task % CV;
      // inputs: 0..3 U, then (MX) 4..8 Q, (IP) 4..11 grad U as [v][d]
      D4 W[4];
      for (int v = 0; v < 4; ++v) {
        W[v] = D4(sh.Wv[qv][v]);
        const int idx = v - NSD * ch;
        if (idx >= 0 && idx < NSD) W[v].d[idx] = 1.0;
      }
      D4 out[4][2];
      if (MX) {
        D4 Qd[5];
        for (int c = 0; c < 5; ++c) {
          Qd[c] = D4(sh.Qv[qv][c]);
          const int idx = 4 + c - NSD * ch;
          if (idx >= 0 && idx < NSD) Qd[c].d[idx] = 1.0;
        }
        vol_point_mx(W, Qd, g, out);
      } else {
        D4 G[4][2];
        for (int v = 0; v < 4; ++v)
          for (int d = 0; d < 2; ++d) {
            G[v][d] = D4(sh.Gv[qv][2 * v + d]);
            const int idx = 4 + 2 * v + d - NSD * ch;
            if (idx >= 0 && idx < NSD) G[v][d].d[idx] = 1.0;
          }
        vol_point_ip(W, G, g, out);
      }
      for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 2; ++d) {
          if (ch == 0) sh.VV[qv][2 * v + d] = out[v][d].v;
          for (int k = 0; k < NSD; ++k) {
            const int col = NSD * ch + k;
            if (col < NIV) jv(qv, 2 * v + d, col) = out[v][d].d[k];
          }
        }
    } else if (task < NQV * CV + 4 * NQ * CF) {
      const int i = task - NQV * CV;
      const int fq = i / CF, ch = i % CF;
      const int f = fq / NQ, q = fq % NQ;
      FaceData fd;
      fd.kind = h.face_kind[4 * p + f];
      fnormal(f, fd.nx, fd.ny);
      fd.tau = tau;
      fd.lf = prm.lf;
      for (int v = 0; v < 4; ++v) fd.uex[v] = sh.uex[f][q][v];
      // inputs: 0..3 U, 4..7 Uhat, then (MX) 8..12 Q, (IP) 8..15 grad U [v][d]
      D4 W[4], Wh[4];
      for (int v = 0; v < 4; ++v) {
        W[v] = D4(sh.Wf[f][q][v]);
        Wh[v] = D4(sh.Wh[f][q][v]);
        int idx = v - NSD * ch;
        if (idx >= 0 && idx < NSD) W[v].d[idx] = 1.0;
        idx = 4 + v - NSD * ch;
        if (idx >= 0 && idx < NSD) Wh[v].d[idx] = 1.0;
      }
      if (MX) {
        D4 Qd[5], s[4], t[4];
        for (int c = 0; c < 5; ++c) {
          Qd[c] = D4(sh.Qf[f][q][c]);
          const int idx = 8 + c - NSD * ch;
          if (idx >= 0 && idx < NSD) Qd[c].d[idx] = 1.0;
        }
        face_point_mx(W, Wh, Qd, fd, g, s, t);
        for (int v = 0; v < 4; ++v) {
          if (ch == 0) { sh.VF[f][q][v] = s[v].v; sh.VF[f][q][4 + v] = t[v].v; }
          for (int k = 0; k < NSD; ++k) {
            const int col = NSD * ch + k;
            if (col < NIF) { jf(f, q, v, col) = s[v].d[k]; jf(f, q, 4 + v, col) = t[v].d[k]; }
          }
        }
      } else {
        D4 G[4][2], s[4], gc[4][2], t[4];
        for (int v = 0; v < 4; ++v)
          for (int d = 0; d < 2; ++d) {
            G[v][d] = D4(sh.Gf[f][q][2 * v + d]);
            const int idx = 8 + 2 * v + d - NSD * ch;
            if (idx >= 0 && idx < NSD) G[v][d].d[idx] = 1.0;
          }
        face_point_ip(W, G, Wh, fd, g, s, gc, t);
        for (int v = 0; v < 4; ++v) {
          if (ch == 0) {
            sh.VF[f][q][v] = s[v].v;
            sh.VF[f][q][4 + 2 * v] = gc[v][0].v;
            sh.VF[f][q][5 + 2 * v] = gc[v][1].v;
            sh.VF[f][q][12 + v] = t[v].v;
          }
          for (int k = 0; k < NSD; ++k) {
            const int col = NSD * ch + k;
            if (col < NIF) {
              jf(f, q, v, col) = s[v].d[k];
              jf(f, q, 4 + 2 * v, col) = gc[v][0].d[k];
              jf(f, q, 5 + 2 * v, col) = gc[v][1].d[k];
              jf(f, q, 12 + v, col) = t[v].d[k];
            }
          }
        }
      }
    } else if (MX) {
      const int il = task - NQV * CV - 4 * NQ * CF;
      const int i = il / CL, lc = il % CL;
      D4 W[4], P[3];
      const double* src = (i < NQV) ? sh.Wv[i] : sh.Wh[(i - NQV) / NQ][(i - NQV) % NQ];
      for (int v = 0; v < 4; ++v) {
        W[v] = D4(src[v]);
        const int idx = v - NSD * lc;
        if (idx >= 0 && idx < NSD) W[v].d[idx] = 1.0;
      }
      lift_point(W, g, P);
      for (int c = 0; c < 3; ++c)
        for (int k = 0; k < NSD; ++k) {
          const int v = NSD * lc + k;
          if (i < NQV) jl(i, c, v) = P[c].d[k];
          else jlf((i - NQV) / NQ, (i - NQV) % NQ, c, v) = P[c].d[k];
        }
    }
  }
  __syncthreads();
  // ---- residual rows ---------------------------------------------------------
  constexpr int NC = S::NC;
  T* bp = blk + (size_t)p * S::BLK;       // row-major NR x NC: [[K C f],[D E h]]
  for (int r = tid; r < NU + NF; r += nt) {
    if (r < NU) {
      const int v = r / NN, n = r % NN, a = n % NP, b = n / NP;
      double acc = 0.0;
      for (int qj = 0; qj < NQ; ++qj)
        for (int qi = 0; qi < NQ; ++qi) {
          const int qv = qi + NQ * qj;
          const double w = tb.W[qi] * tb.W[qj] * jac;
          acc += w * (sh.VV[qv][2 * v] * tb.D[qi][a] * tb.L[qj][b] * sx +
                      sh.VV[qv][2 * v + 1] * tb.L[qi][a] * tb.D[qj][b] * sy);
        }
      for (int f = 0; f < 4; ++f) {
        const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
        for (int q = 0; q < NQ; ++q) {
          double ph, pxi, peta;
          face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
          const double w = tb.W[q] * wl;
          acc += w * sh.VF[f][q][v] * ph;
          if (!MX) acc += w * (sh.VF[f][q][4 + 2 * v] * pxi * sx + sh.VF[f][q][5 + 2 * v] * peta * sy);
        }
      }
      const double mass = tb.NW[a] * tb.NW[b] * jac;
      const size_t gi = (size_t)e * NU + r;
      if (Rh) Rh[gi] = acc;
      bp[(size_t)r * NC + NC - 1] = static_cast<T>(mass * sh.U[r] + dta * acc - (rhs ? rhs[gi] : 0.0));
    } else {
      const int rr = r - NU, f = rr / NFF, v = (rr % NFF) / NP, mm = rr % NP;
      const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
      constexpr int TO = MX ? 4 : 12;
      double acc = 0.0;
      for (int q = 0; q < NQ; ++q) acc += tb.W[q] * wl * tb.L[q][mm] * sh.VF[f][q][TO + v];
      // the element's share of its facet residuals: large where the two sides cancel,
      // so it is kept in FP64 (hres) and the augmented column starts from 0
      bp[(size_t)(NU + rr) * NC + NC - 1] = T(0);
      hres[(size_t)p * NF + rr] = acc;
    }
  }
  if constexpr (!JAC) return;
  // the point-wise Jacobians are in the record; the block contraction kernels read them
}

// ---------------------------------------------------------------------------
// Element block contraction from the point records (sum factorisation).
//
// Volume contributions to K = M + dt_a dR/dU, A12 = dt_a dR/dQ and the lifting
// block A21 = M_Q^-1 dl/dU all have the form
//   sum_{qi,qj} w_i w_j |J| [ s_x D(qi,a) L(qj,b) Jx(qi,qj) + s_y L(qi,a) D(qj,b) Jy(qi,qj) ] L(qi,a2) L(qj,b2)
// for row node (a, b) and column node (a2, b2).  One thread owns the row/column
// pair and the node pair (a, a2) and keeps all (b, b2) in registers: the qi sum
// is done once per qj, the qj sum as a rank-2 update of the 25 accumulators
// with the 1D tables TLL[q][b][b2] = w_q L(q,b) L(q,b2), TDL = w_q D(q,b) L(q,b2).
// Faces x-/x+ add LE(a) LE(a2) sum_q TLL[q][b][b2] J_f(q), faces y-/y+ add
// LE(b) LE(b2) sum_q TLL[q][a][a2] J_f(q).  The face-only blocks C, D, E, A32,
// A23 are an edge value times one 1D sum per entry; the distinct sums are
// tabulated first.
//
// Work split: five workgroups per HDG-MX element (K | A12 | A21 | C D E |
// A32 A23), two per inviscid HDG-IP element (K | C D E), numbered so that the
// workgroups of one element run on the same XCD and share its L2 copy of the
// point record.
// ---------------------------------------------------------------------------
template <int K, class T> struct CtShared {
  static constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NQV = NQ * NQ;
  T TLL[NQ][NP][NP];
  T TDL[NQ][NP][NP];
  T LE[2][NP];
  T NW[NP];
  union {
    struct {                     // groups 0-2: up to 20 (row variable, column variable) pairs
      T JX[20][NQV];
      T JY[20][NQV];
      T JS[20][4][NQ];
    } v;
    struct {                     // groups 3-4: staged face records and their line sums
      T JF[4][NQ][8][8];
      T JLF[4][NQ][3][4];
      T G[80 * NP * NP];
    } f;
  } u;
};

// The same 1D tables W L L and W D L in constant memory.  In the rank-2 updates
// every lane of a wave reads the same entry, so the contraction takes them
// through scalar loads as instruction operands instead of LDS broadcasts (which
// cost as much LDS bandwidth as a full-width read).  One copy per degree and
// storage type, written once per device by ct_upload.
template <int K, class T> struct CtTab {
  static constexpr int NP = K + 1, NQ = (3 * K + 2) / 2;
  T TLL[NQ][NP][NP];
  T TDL[NQ][NP][NP];
};
template <int K, class T> struct CtSym;
#define CT_SYM(KK, TT, NAME)                                                                        \
  __constant__ CtTab<KK, TT> NAME;                                                                  \
  template <> struct CtSym<KK, TT> {                                                                \
    static __device__ __forceinline__ const CtTab<KK, TT>& get() { return NAME; }                   \
    static const void* symbol() { return reinterpret_cast<const void*>(&HIP_SYMBOL(NAME)); }        \
  };
CT_SYM(1, float, ct_tab_1f)
CT_SYM(2, float, ct_tab_2f)
CT_SYM(3, float, ct_tab_3f)
CT_SYM(4, float, ct_tab_4f)
CT_SYM(1, double, ct_tab_1d)
CT_SYM(2, double, ct_tab_2d)
CT_SYM(3, double, ct_tab_3d)
CT_SYM(4, double, ct_tab_4d)
#undef CT_SYM

template <int K, class T> static hipError_t ct_upload_one(const BasisTable& tb) {
  using C = CtTab<K, T>;
  C h;
  for (int q = 0; q < C::NQ; ++q)
    for (int a = 0; a < C::NP; ++a)
      for (int a2 = 0; a2 < C::NP; ++a2) {
        h.TLL[q][a][a2] = static_cast<T>(tb.W[q] * tb.L[q][a] * tb.L[q][a2]);
        h.TDL[q][a][a2] = static_cast<T>(tb.W[q] * tb.D[q][a] * tb.L[q][a2]);
      }
  return hipMemcpyToSymbol(CtSym<K, T>::symbol(), &h, sizeof(h), 0, hipMemcpyHostToDevice);
}

// fills the constant tables of degree K (both storage types) on the current device,
// once per device and degree
static hipError_t ct_upload(int K, const BasisTable& tb) {
  static std::mutex mu;
  static std::vector<unsigned> done;   // per device: bit K
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, 0u);
  if (done[dev] & (1u << K)) return hipSuccess;
  switch (K) {
    case 1: e = ct_upload_one<1, float>(tb); if (e == hipSuccess) e = ct_upload_one<1, double>(tb); break;
    case 2: e = ct_upload_one<2, float>(tb); if (e == hipSuccess) e = ct_upload_one<2, double>(tb); break;
    case 3: e = ct_upload_one<3, float>(tb); if (e == hipSuccess) e = ct_upload_one<3, double>(tb); break;
    case 4: e = ct_upload_one<4, float>(tb); if (e == hipSuccess) e = ct_upload_one<4, double>(tb); break;
    default: return hipErrorInvalidValue;
  }
  if (e == hipSuccess) done[dev] |= 1u << K;
  return e;
}

// coefficients of the lifted primitives in the mixed equations: component c of
// l(U, Uhat) = sum_p (cx[c][p] d/dx + cy[c][p] d/dy) of P_p, P = (u, v, theta)
template <class T>
__device__ __forceinline__ void lift_coef(int c, T cx[3], T cy[3]) {
  cx[0] = cx[1] = cx[2] = cy[0] = cy[1] = cy[2] = T(0);
  switch (c) {
    case 0: cx[0] = T(2.0 / 3.0); cy[1] = T(-1.0 / 3.0); break;    // eps_11 - tr/3
    case 1: cx[1] = T(1); cy[0] = T(1); break;                 // 2 eps_12 (weighted by 2 in M_Q)
    case 2: cx[0] = T(-1.0 / 3.0); cy[1] = T(2.0 / 3.0); break;    // eps_22 - tr/3
    case 3: cx[2] = T(1); break;                              // grad theta, x
    default: cy[2] = T(1); break;                             // grad theta, y
  }
}

// waves per SIMD the contraction's registers are held to (it is latency-bound: 8 measured
// faster than the unconstrained 4)
#ifndef CT_WAVES_PER_EU
#define CT_WAVES_PER_EU 8
#endif
#if CT_WAVES_PER_EU > 0
#define CT_WAVES __attribute__((amdgpu_waves_per_eu(CT_WAVES_PER_EU, CT_WAVES_PER_EU)))
#else
#define CT_WAVES
#endif
template <int K, class T, bool MX>
__global__ void __launch_bounds__(256) CT_WAVES hdg_contract_kernel(DeviceMesh m, DeviceHDG h, double dt_a,
                                                           const double* __restrict__ rec,
                                                           T* __restrict__ blk, T* __restrict__ scr) {
  using S = HS<K, true>;
  using R = PointRec<K, MX>;
  constexpr int NGRP = MX ? 5 : 2;              // HDG-IP: K and the face-only blocks C D E
  constexpr int NP = S::NP, NQ = S::NQ, NN = S::NN, NQV = S::NQV, NU = S::NU, NF = S::NF, NFF = S::NFF;
  constexpr int NQM = S::NQM, NR = S::NR, NC = S::NC;
  __shared__ CtShared<K, T> sh;
  // XCD-aware numbering: consecutive workgroups go to consecutive XCDs, so the
  // five groups of element p are spread over blocks 8 apart
  const int L = blockIdx.x;
  const int xcd = L & 7, rr = L >> 3;
  const int grp = MX ? rr % NGRP : (rr % NGRP == 0 ? 0 : 3);
  const int p = 8 * (rr / NGRP) + xcd;
  if (p >= h.n_im) return;
  const int e = h.im_list[p];
  const int tid = threadIdx.x, nt = blockDim.x;
  const BasisTable& tb = *m.tab;
  const double hx = m.hx[e], hy = m.hy[e];
  const T sx = T(2.0 / hx), sy = T(2.0 / hy), jac = T(0.25 * hx * hy);
  const T wlx = T(0.5 * hy), wly = T(0.5 * hx);     // line measure factor of x-faces / y-faces
  const T dta = T(dt_a * elem_dt(m, e));
  for (int i = tid; i < NQ * NN; i += nt) {
    const int q = i / NN, a = (i / NP) % NP, a2 = i % NP;
    sh.TLL[q][a][a2] = tb.W[q] * tb.L[q][a] * tb.L[q][a2];
    sh.TDL[q][a][a2] = tb.W[q] * tb.D[q][a] * tb.L[q][a2];
  }
  if (tid < 2 * NP) sh.LE[tid / NP][tid % NP] = tb.LE[tid / NP][tid % NP];
  if (tid < NP) sh.NW[tid] = tb.NW[tid];
  const double* rp = rec + (size_t)p * R::SIZE;
  T* bp = blk + (size_t)p * S::BLK;
  T* Lm = scr + (size_t)p * S::SCR;             // [A12; A32]      NR x NQM
  T* Rm = Lm + (size_t)NR * NQM;                // M_Q^-1 [A21 A23] NQM x NR
  if (grp <= 2) {
    // gather the pair slices: grp 0 K (v, v2), grp 1 A12 (v, c), grp 2 A21 (c, v2)
    const int npair = (grp == 0) ? 16 : 20;
    for (int i = tid; i < npair * NQV; i += nt) {
      const int pr = i / NQV, qv = i % NQV;
      T jx, jy;
      if (grp == 0) {
        const int v = pr >> 2, v2 = pr & 3;
        jx = rp[R::JV + (qv * 8 + 2 * v) * R::NIV + v2];
        jy = rp[R::JV + (qv * 8 + 2 * v + 1) * R::NIV + v2];
      } else if (grp == 1) {
        const int v = pr / 5, c = pr % 5;
        jx = rp[R::JV + (qv * 8 + 2 * v) * 9 + 4 + c];
        jy = rp[R::JV + (qv * 8 + 2 * v + 1) * 9 + 4 + c];
      } else {
        const int c = pr >> 2, v2 = pr & 3;
        T cx[3], cy[3];
        lift_coef(c, cx, cy);
        jx = jy = 0.0;
        for (int pp = 0; pp < 3; ++pp) {
          const T d = rp[R::JL + (qv * 3 + pp) * 4 + v2];
          jx += cx[pp] * d;
          jy += cy[pp] * d;
        }
      }
      sh.u.v.JX[pr][qv] = jx;
      sh.u.v.JY[pr][qv] = jy;
    }
    if (grp < 2)
      for (int i = tid; i < npair * 4 * NQ; i += nt) {
        const int pr = i / (4 * NQ), f = (i / NQ) % 4, q = i % NQ;
        const int v = (grp == 0) ? pr >> 2 : pr / 5;
        const int col = (grp == 0) ? (pr & 3) : 8 + pr % 5;
        sh.u.v.JS[pr][f][q] = rp[R::JF + ((f * NQ + q) * R::NOF + v) * R::NIF + col];
      }
    __syncthreads();
    const T cx = jac * sx, cy = jac * sy;
    for (int t = tid; t < npair * NN; t += nt) {
      const int pr = t / NN, a = (t / NP) % NP, a2 = t % NP;
      T acc[NP][NP];
#pragma unroll
      for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int b2 = 0; b2 < NP; ++b2) acc[b][b2] = 0.0;
      const T* jxp = sh.u.v.JX[pr];
      const T* jyp = sh.u.v.JY[pr];
      const CtTab<K, T>& ct = CtSym<K, T>::get();
#pragma unroll 1
      for (int qj = 0; qj < NQ; ++qj) {
        T px = 0.0, py = 0.0;
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
          px += sh.TDL[qi][a][a2] * jxp[qi + NQ * qj];
          py += sh.TLL[qi][a][a2] * jyp[qi + NQ * qj];
        }
        px *= cx;
        py *= cy;
#pragma unroll
        for (int b = 0; b < NP; ++b)
#pragma unroll
          for (int b2 = 0; b2 < NP; ++b2) {
            acc[b][b2] += ct.TLL[qj][b][b2] * px;
            acc[b][b2] += ct.TDL[qj][b][b2] * py;
          }
      }
      if (grp < 2) {
        const T(*js)[NQ] = sh.u.v.JS[pr];
#pragma unroll 1
        for (int s = 0; s < 2; ++s) {       // x-faces: f = s
          const T c0 = wlx * sh.LE[s][a] * sh.LE[s][a2];
#pragma unroll 1
          for (int q = 0; q < NQ; ++q) {
            const T cq = c0 * js[s][q];
#pragma unroll
            for (int b = 0; b < NP; ++b)
#pragma unroll
              for (int b2 = 0; b2 < NP; ++b2) acc[b][b2] += ct.TLL[q][b][b2] * cq;
          }
        }
#pragma unroll 1
        for (int s = 0; s < 2; ++s) {       // y-faces: f = 2 + s
          T sg = 0.0;
#pragma unroll
          for (int q = 0; q < NQ; ++q) sg += sh.TLL[q][a][a2] * js[2 + s][q];
          sg *= wly;
#pragma unroll
          for (int b = 0; b < NP; ++b)
#pragma unroll
            for (int b2 = 0; b2 < NP; ++b2) acc[b][b2] += sh.LE[s][b] * sh.LE[s][b2] * sg;
        }
      }
      if (grp == 0) {
        const int v = pr >> 2, v2 = pr & 3;
#pragma unroll
        for (int b = 0; b < NP; ++b)
#pragma unroll
          for (int b2 = 0; b2 < NP; ++b2) {
            const int row = v * NN + a + NP * b, col = v2 * NN + a2 + NP * b2;
            const T mass = (row == col) ? sh.NW[a] * sh.NW[b] * jac : T(0);
            bp[(size_t)row * NC + col] = dta * acc[b][b2] + mass;
          }
      } else if (grp == 1) {
        const int v = pr / 5, c = pr % 5;
#pragma unroll
        for (int b = 0; b < NP; ++b)
#pragma unroll
          for (int b2 = 0; b2 < NP; ++b2)
            Lm[(size_t)(v * NN + a + NP * b) * NQM + c * NN + a2 + NP * b2] = dta * acc[b][b2];
      } else {
        const int c = pr >> 2, v2 = pr & 3;
        const T fc = (c == 1) ? T(2) : T(1);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          const T minv = T(1) / (fc * sh.NW[a] * sh.NW[b] * jac);
#pragma unroll
          for (int b2 = 0; b2 < NP; ++b2) Rm[(size_t)(c * NN + a + NP * b) * NR + v2 * NN + a2 + NP * b2] = minv * acc[b][b2];
        }
      }
    }
    return;
  }
  // Face-only blocks.  Each entry is an edge value of a basis function times a line sum
  //   G(x, y) = sum_q w_q L(q, x) L(q, y) J(q)
  // over one face, and the sums depend on five of the entry's indices only, so each is
  // formed once into LDS and the blocks are then written from those tables by threads
  // that own one column each (consecutive lanes write consecutive addresses of a row).
  // Staged face Jacobians JF[f][q][r][c]: group 3 takes rows s (0..3) and t (4..7) with
  // columns U (0..3) and Uhat (4..7); group 4 takes the t rows (0..3) with the Q columns
  // (0..4), and the lifting traces JLF.
  if (grp == 3) {
    for (int i = tid; i < 4 * NQ * 64; i += nt) {
      const int fq = i / 64, r = (i / 8) % 8, col = i % 8;
      const int src = r < 4 ? r : R::TO + (r - 4);
      (&sh.u.f.JF[0][0][0][0])[i] = rp[R::JF + (fq * R::NOF + src) * R::NIF + col];
    }
  } else if constexpr (MX) {
    for (int i = tid; i < 4 * NQ * 20; i += nt) {
      const int fq = i / 20, v = (i % 20) / 5, c = i % 5;
      (&sh.u.f.JF[0][0][0][0])[fq * 64 + v * 8 + c] = rp[R::JF + (fq * R::NOF + R::TO + v) * R::NIF + 8 + c];
    }
    for (int i = tid; i < 4 * NQ * 12; i += nt) (&sh.u.f.JLF[0][0][0][0])[i] = rp[R::JLF + i];
  }
  T* G = sh.u.f.G;
  // G[((f * 4 + v) * NV2 + v2) * NN + x * NP + y] = sum_q TLL[q][x][y] JF[f][q][r0 + v][c0 + v2].
  // A thread keeps one node pair (x, y), with its NQ table entries in registers, and
  // forms the sums of several (f, v, v2).
  auto line_sums = [&](auto nv2, int r0, int c0) {
    constexpr int NV2 = decltype(nv2)::value;
    const int TPX = nt / NN, xy = tid % NN, sl = tid / NN;
    if (sl >= TPX) return;
    const int x = xy / NP, y = xy % NP;
    T tl[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) tl[q] = sh.TLL[q][x][y];
    for (int fvv = sl; fvv < 16 * NV2; fvv += TPX) {
      const int v2 = fvv % NV2, fv = fvv / NV2;
      const T* j = &sh.u.f.JF[fv >> 2][0][r0 + (fv & 3)][c0 + v2];
      T acc = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc += tl[q] * j[q * 64];
      G[fvv * NN + xy] = acc;
    }
  };
  // Rows of the facet side (f, v, mm) against a column of the element side (w, a2, b2) with
  // NW line sums per face row: a thread owns the column and takes whole (f, v) row groups,
  // the NP rows mm of a group unrolled.  Entry = edge value of the column's basis function
  // on face f (LE(s, a2) on x-faces, LE(s, b2) on y-faces) times the line sum over (mm, the
  // other index).  Writes dst[(row0 + row) * ld + col].
  auto face_rows = [&](auto nw, T* dst, int ld, int row0) {
    constexpr int NW = decltype(nw)::value, NCOL = NW * NN;
    const int lanes = nt / NCOL, lane = tid / NCOL, col = tid % NCOL;
    if (lane >= lanes) return;
    const int w = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
    const T ex0 = wlx * sh.LE[0][a2], ex1 = wlx * sh.LE[1][a2];
    const T ey0 = wly * sh.LE[0][b2], ey1 = wly * sh.LE[1][b2];
    for (int fv = lane; fv < 16; fv += lanes) {
      const int f = fv >> 2;
      const T e = f == 0 ? ex0 : (f == 1 ? ex1 : (f == 2 ? ey0 : ey1));
      const T* g = G + (fv * NW + w) * NN + (f < 2 ? b2 : a2);
      T* d = dst + (size_t)(row0 + fv * NP) * ld + col;
#pragma unroll
      for (int mm = 0; mm < NP; ++mm) d[(size_t)mm * ld] = e * g[mm * NP];
    }
  };
  if (grp == 3) {
    // C = dt_a dR/dUhat (NU x NF): row (v, b, a), column (f, v2, m2); the x-faces pair
    // LE(a) with the line sum over (b, m2), the y-faces LE(b) with the sum over (a, m2).
    // A thread owns the column and takes whole (v, b) row groups, the rows a unrolled.
    __syncthreads();
    line_sums(std::integral_constant<int, 4>{}, 0, 4);
    __syncthreads();
    {
      const int lanes = nt / NF, lane = tid / NF, col = tid % NF;
      if (lane < lanes) {
        const int f = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP, s = f & 1;
        const bool xf = f < 2;
        const T sc = dta * (xf ? wlx : wly);
        T le[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) le[a] = sc * sh.LE[s][a];
        const T* g = G + (f * 16 + v2) * NN + m2;
        for (int vb = lane; vb < 4 * NP; vb += lanes) {
          const int v = vb / NP, b = vb % NP;
          const T lb = sc * sh.LE[s][b];
          const T* gv = g + v * 4 * NN;
          T* d = bp + (size_t)(v * NN + b * NP) * NC + NU + col;
#pragma unroll
          for (int a = 0; a < NP; ++a)
            d[(size_t)a * NC] = xf ? le[a] * gv[b * NP] : lb * gv[a * NP];
        }
      }
    }
    // D = dh/dU (NF x NU): row (f, v, mm), column (v2, b2, a2)
    __syncthreads();
    line_sums(std::integral_constant<int, 4>{}, 4, 0);
    __syncthreads();
    face_rows(std::integral_constant<int, 4>{}, bp, NC, NU);
    // E = dh/dUhat (NF x NF, block diagonal over the faces): row (f, v, mm), column (f2, v2, m2)
    __syncthreads();
    line_sums(std::integral_constant<int, 4>{}, 4, 4);
    __syncthreads();
    {
      const int lanes = nt / NF, lane = tid / NF, col = tid % NF;
      if (lane < lanes) {
        const int f2 = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP;
        const T wl = (f2 < 2) ? wlx : wly;
        for (int fv = lane; fv < 16; fv += lanes) {
          const int f = fv >> 2;
          const bool on = f == f2;
          const T* g = G + (fv * 4 + v2) * NN + m2;
          T* d = bp + (size_t)(NU + fv * NP) * NC + NU + col;
#pragma unroll
          for (int mm = 0; mm < NP; ++mm) d[(size_t)mm * NC] = on ? wl * g[mm * NP] : T(0);
        }
      }
    }
    return;
  }
  if constexpr (MX) {
    // A32 = dh/dQ (NF x NQM, rows NU.. of Lm): row (f, v, mm), column (c, b2, a2)
    __syncthreads();
    line_sums(std::integral_constant<int, 5>{}, 0, 0);
    __syncthreads();
    face_rows(std::integral_constant<int, 5>{}, Lm, NQM, NU);
    // A23 = M_Q^-1 dl/dUhat (NQM x NF, columns NU.. of Rm): row (c, b, a), column (f, v2, m2).
    // The line sums take the lifted normal traces g_q = sum_p cn_p JLF[f][q][p][v2] with
    // cn_p = cx_p n_x + cy_p n_y of component c (tabulated first):
    // G[((f * 5 + c) * 4 + v2) * NN + x * NP + y] = sum_q TLL[q][x][y] g_q
    __shared__ T CN[4][5][3];
    if (tid < 20) {
      const int f = tid / 5, c = tid % 5;
      double nxd, nyd;
      fnormal(f, nxd, nyd);
      T cx[3], cy[3];
      lift_coef(c, cx, cy);
      for (int pp = 0; pp < 3; ++pp) CN[f][c][pp] = cx[pp] * T(nxd) + cy[pp] * T(nyd);
    }
    __syncthreads();
    {
      const int TPX = nt / NN, xy = tid % NN, sl = tid / NN;
      if (sl < TPX) {
        const int x = xy / NP, y = xy % NP;
        T tl[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) tl[q] = sh.TLL[q][x][y];
        for (int fcv = sl; fcv < 80; fcv += TPX) {
          const int v2 = fcv % 4, c = (fcv / 4) % 5, f = fcv / 20;
          const T c0 = CN[f][c][0], c1 = CN[f][c][1], c2 = CN[f][c][2];
          T acc = 0.0;
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            acc += tl[q] * (c0 * sh.u.f.JLF[f][q][0][v2] + c1 * sh.u.f.JLF[f][q][1][v2] +
                            c2 * sh.u.f.JLF[f][q][2][v2]);
          G[fcv * NN + xy] = acc;
        }
      }
    }
    __syncthreads();
    {
      const int lanes = nt / NF, lane = tid / NF, col = tid % NF;
      if (lane < lanes) {
        const int f = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP, s = f & 1;
        const bool xf = f < 2;
        const T wl = xf ? wlx : wly;
        T le[NP], mw[NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          le[a] = wl * sh.LE[s][a];
          mw[a] = T(1) / (sh.NW[a] * jac);
        }
        for (int cb = lane; cb < 5 * NP; cb += lanes) {
          const int c = cb / NP, b = cb % NP;
          const T lb = wl * sh.LE[s][b];
          // -M_Q^-1 on row (c, a, b): M_Q is diagonal, NW(a) NW(b) |J| (twice that for c = 1)
          const T mb = -((c == 1) ? T(0.5) : T(1)) / sh.NW[b];
          const T* g = G + ((f * 5 + c) * 4 + v2) * NN + m2;
          T* d = Rm + (size_t)(c * NN + b * NP) * NR + NU + col;
#pragma unroll
          for (int a = 0; a < NP; ++a)
            d[(size_t)a * NR] = mb * mw[a] * (xf ? le[a] * g[b * NP] : lb * g[a * NP]);
        }
      }
    }
  }
}

// Viscous HDG-IP: the same contraction of the point records into K, C, D, E, with the
// gradient columns and rows the viscous flux brings (Sec. 3.4): volume terms pair a test
// derivative with a trial value or derivative, face terms pair test value/derivatives
// with trial value/derivatives.  Every term is a product of 1D factors, so each is a sum
// over one quadrature direction of the tabulated products W L L, W D L, W L D, W D D.
// Three workgroups per element: K rows of v in {0, 1}, K rows of v in {2, 3}, and C D E.
template <int K, class T> struct CtIpShared {
  static constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NQV = NQ * NQ;
  T TLL[NQ][NP][NP], TDL[NQ][NP][NP], TLD[NQ][NP][NP], TDD[NQ][NP][NP];
  T LE[2][NP], DE[2][NP], NW[NP];
  union {
    struct {
      T J[8][6][NQV];               // per (v, v2) pair: d(F_x, F_y)_v / d(U, U_x, U_y)_v2 at volume points
      T JS[8][4][NQ][9];            // per pair and face point: rows (s, g_x, g_y) x columns (U, U_x, U_y)
    } v;
    struct {
      T JF[4][NQ][16][16];          // face records: rows s, g, t; columns U, Uhat, grad U
    } f;
  } u;
};

template <int K, class T>
__global__ void __launch_bounds__(256) hdg_contract_ipv_kernel(DeviceMesh m, DeviceHDG h, double dt_a,
                                                               const double* __restrict__ rec, T* __restrict__ blk) {
  using S = HS<K, false>;
  using R = PointRec<K, false>;
  constexpr int NP = S::NP, NQ = S::NQ, NN = S::NN, NQV = S::NQV, NU = S::NU, NF = S::NF, NFF = S::NFF;
  constexpr int NC = S::NC;
  static_assert(R::NOF == 16 && R::NIF == 16 && R::NIV == 12 && R::TO == 12, "viscous HDG-IP record layout");
  __shared__ CtIpShared<K, T> sh;
  const int grp = blockIdx.x % 3, p = blockIdx.x / 3;
  if (p >= h.n_im) return;
  const int e = h.im_list[p];
  const int tid = threadIdx.x, nt = blockDim.x;
  const BasisTable& tb = *m.tab;
  const double hx = m.hx[e], hy = m.hy[e];
  const T sx = T(2.0 / hx), sy = T(2.0 / hy), jac = T(0.25 * hx * hy);
  const T wlx = T(0.5 * hy), wly = T(0.5 * hx);
  const T dta = T(dt_a * elem_dt(m, e));
  for (int i = tid; i < NQ * NN; i += nt) {
    const int q = i / NN, x = (i / NP) % NP, y = i % NP;
    sh.TLL[q][x][y] = T(tb.W[q] * tb.L[q][x] * tb.L[q][y]);
    sh.TDL[q][x][y] = T(tb.W[q] * tb.D[q][x] * tb.L[q][y]);
    sh.TLD[q][x][y] = T(tb.W[q] * tb.L[q][x] * tb.D[q][y]);
    sh.TDD[q][x][y] = T(tb.W[q] * tb.D[q][x] * tb.D[q][y]);
  }
  if (tid < 2 * NP) {
    sh.LE[tid / NP][tid % NP] = T(tb.LE[tid / NP][tid % NP]);
    sh.DE[tid / NP][tid % NP] = T(tb.DE[tid / NP][tid % NP]);
  }
  if (tid < NP) sh.NW[tid] = T(tb.NW[tid]);
  const double* rp = rec + (size_t)p * R::SIZE;
  T* bp = blk + (size_t)p * S::BLK;
  if (grp < 2) {
    // pairs pr = 4 vl + v2 with the row variable v = 2 grp + vl
    for (int i = tid; i < 8 * NQV; i += nt) {
      const int pr = i / NQV, qv = i % NQV, v = 2 * grp + pr / 4, v2 = pr % 4;
      const double* jx = rp + R::JV + ((size_t)qv * 8 + 2 * v) * R::NIV;
      const double* jy = jx + R::NIV;
      sh.u.v.J[pr][0][qv] = T(jx[v2]);
      sh.u.v.J[pr][1][qv] = T(jx[4 + 2 * v2]);
      sh.u.v.J[pr][2][qv] = T(jx[5 + 2 * v2]);
      sh.u.v.J[pr][3][qv] = T(jy[v2]);
      sh.u.v.J[pr][4][qv] = T(jy[4 + 2 * v2]);
      sh.u.v.J[pr][5][qv] = T(jy[5 + 2 * v2]);
    }
    for (int i = tid; i < 8 * 4 * NQ * 9; i += nt) {
      const int pr = i / (4 * NQ * 9), f = (i / (NQ * 9)) % 4, q = (i / 9) % NQ, k = i % 9;
      const int v = 2 * grp + pr / 4, v2 = pr % 4;
      const int ri = k / 3, ci = k % 3;
      const int row = ri == 0 ? v : (ri == 1 ? 4 + 2 * v : 5 + 2 * v);
      const int col = ci == 0 ? v2 : (ci == 1 ? 8 + 2 * v2 : 9 + 2 * v2);
      sh.u.v.JS[pr][f][q][k] = T(rp[R::JF + (((size_t)f * NQ + q) * R::NOF + row) * R::NIF + col]);
    }
    __syncthreads();
    for (int t = tid; t < 8 * NN; t += nt) {
      const int pr = t / NN, a = (t / NP) % NP, a2 = t % NP;
      const int v = 2 * grp + pr / 4, v2 = pr % 4;
      T acc[NP][NP];
#pragma unroll
      for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int b2 = 0; b2 < NP; ++b2) acc[b][b2] = T(0);
      // volume: (test d/dx, d/dy) x (trial value, d/dx, d/dy)
      const T(*J)[NQV] = sh.u.v.J[pr];
#pragma unroll 1
      for (int qj = 0; qj < NQ; ++qj) {
        T s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
#pragma unroll
        for (int qi = 0; qi < NQ; ++qi) {
          const int qv = qi + NQ * qj;
          s0 += sh.TDL[qi][a][a2] * J[0][qv];
          s1 += sh.TDD[qi][a][a2] * J[1][qv];
          s2 += sh.TDL[qi][a][a2] * J[2][qv];
          s3 += sh.TLL[qi][a][a2] * J[3][qv];
          s4 += sh.TLD[qi][a][a2] * J[4][qv];
          s5 += sh.TLL[qi][a][a2] * J[5][qv];
        }
        const T cLL = jac * sx * (s0 + sx * s1), cLD = jac * sx * sy * s2;
        const T cDL = jac * sy * (s3 + sx * s4), cDD = jac * sy * sy * s5;
#pragma unroll
        for (int b = 0; b < NP; ++b)
#pragma unroll
          for (int b2 = 0; b2 < NP; ++b2)
            acc[b][b2] += sh.TLL[qj][b][b2] * cLL + sh.TLD[qj][b][b2] * cLD + sh.TDL[qj][b][b2] * cDL +
                          sh.TDD[qj][b][b2] * cDD;
      }
      // x-faces (f = s): test and trial factors along x are edge values LE / derivatives DE
#pragma unroll 1
      for (int s = 0; s < 2; ++s) {
        const T La = sh.LE[s][a], Da = sh.DE[s][a], La2 = sh.LE[s][a2], Da2 = sh.DE[s][a2];
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
          const T* j = sh.u.v.JS[pr][s][q];
          const T cLL = wlx * (La * La2 * j[0] + sx * (La * Da2 * j[1] + Da * La2 * j[3]) + sx * sx * Da * Da2 * j[4]);
          const T cLD = wlx * sy * (La * La2 * j[2] + sx * Da * La2 * j[5]);
          const T cDL = wlx * sy * (La * La2 * j[6] + sx * La * Da2 * j[7]);
          const T cDD = wlx * sy * sy * La * La2 * j[8];
#pragma unroll
          for (int b = 0; b < NP; ++b)
#pragma unroll
            for (int b2 = 0; b2 < NP; ++b2)
              acc[b][b2] += sh.TLL[q][b][b2] * cLL + sh.TLD[q][b][b2] * cLD + sh.TDL[q][b][b2] * cDL +
                            sh.TDD[q][b][b2] * cDD;
        }
      }
      // y-faces (f = 2 + s): the quadrature runs along x (a, a2), the edge factors along y
#pragma unroll 1
      for (int s = 0; s < 2; ++s) {
        const T(*js)[9] = sh.u.v.JS[pr][2 + s];
        T S0 = 0, S1 = 0, S2 = 0, S3 = 0, S4 = 0, S5 = 0, S6 = 0, S7 = 0, S8 = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const T ll = sh.TLL[q][a][a2], ld = sh.TLD[q][a][a2], dl = sh.TDL[q][a][a2], dd = sh.TDD[q][a][a2];
          S0 += ll * js[q][0];
          S1 += ld * js[q][1];
          S2 += ll * js[q][2];
          S3 += dl * js[q][3];
          S4 += dd * js[q][4];
          S5 += dl * js[q][5];
          S6 += ll * js[q][6];
          S7 += ld * js[q][7];
          S8 += ll * js[q][8];
        }
        const T cEE = wly * (S0 + sx * (S1 + S3) + sx * sx * S4);
        const T cED = wly * sy * (S2 + sx * S5);
        const T cDE = wly * sy * (S6 + sx * S7);
        const T cDD = wly * sy * sy * S8;
#pragma unroll
        for (int b = 0; b < NP; ++b)
#pragma unroll
          for (int b2 = 0; b2 < NP; ++b2)
            acc[b][b2] += sh.LE[s][b] * (sh.LE[s][b2] * cEE + sh.DE[s][b2] * cED) +
                          sh.DE[s][b] * (sh.LE[s][b2] * cDE + sh.DE[s][b2] * cDD);
      }
#pragma unroll
      for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int b2 = 0; b2 < NP; ++b2) {
          const int row = v * NN + a + NP * b, col = v2 * NN + a2 + NP * b2;
          const T mass = (row == col) ? sh.NW[a] * sh.NW[b] * jac : T(0);
          bp[(size_t)row * NC + col] = dta * acc[b][b2] + mass;
        }
    }
    return;
  }
  // C = dt_a dR/dUhat, D = dh/dU, E = dh/dUhat from the face records
  for (int i = tid; i < 4 * NQ * 16 * 16; i += nt) (&sh.u.f.JF[0][0][0][0])[i] = T(rp[R::JF + i]);
  __syncthreads();
  auto fs = [&](const T(*tab)[NP][NP], int f, int x, int y, int r, int c) {
    T acc = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc += tab[q][x][y] * sh.u.f.JF[f][q][r][c];
    return acc;
  };
  constexpr int NCC = NU * NF, NDD = NF * NU, NEE = NF * NF;
  for (int i = tid; i < NCC + NDD + NEE; i += nt) {
    if (i < NCC) {
      const int row = i / NF, col = i % NF;
      const int v = row / NN, n = row % NN, a = n % NP, b = n / NP;
      const int f = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP, s = f & 1, c = 4 + v2;
      T val;
      if (f < 2)
        val = wlx * (sh.LE[s][a] * fs(sh.TLL, f, b, m2, v, c) + sx * sh.DE[s][a] * fs(sh.TLL, f, b, m2, 4 + 2 * v, c) +
                     sy * sh.LE[s][a] * fs(sh.TDL, f, b, m2, 5 + 2 * v, c));
      else
        val = wly * (sh.LE[s][b] * fs(sh.TLL, f, a, m2, v, c) + sx * sh.LE[s][b] * fs(sh.TDL, f, a, m2, 4 + 2 * v, c) +
                     sy * sh.DE[s][b] * fs(sh.TLL, f, a, m2, 5 + 2 * v, c));
      bp[(size_t)row * NC + NU + col] = dta * val;
    } else if (i < NCC + NDD) {
      const int j = i - NCC, row = j / NU, col = j % NU;
      const int f = row / NFF, v = (row % NFF) / NP, mm = row % NP, s = f & 1, r = 12 + v;
      const int v2 = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
      T val;
      if (f < 2)
        val = wlx * (sh.LE[s][a2] * fs(sh.TLL, f, mm, b2, r, v2) + sx * sh.DE[s][a2] * fs(sh.TLL, f, mm, b2, r, 8 + 2 * v2) +
                     sy * sh.LE[s][a2] * fs(sh.TLD, f, mm, b2, r, 9 + 2 * v2));
      else
        val = wly * (sh.LE[s][b2] * fs(sh.TLL, f, mm, a2, r, v2) + sx * sh.LE[s][b2] * fs(sh.TLD, f, mm, a2, r, 8 + 2 * v2) +
                     sy * sh.DE[s][b2] * fs(sh.TLL, f, mm, a2, r, 9 + 2 * v2));
      bp[(size_t)(NU + row) * NC + col] = val;
    } else {
      const int j = i - NCC - NDD, row = j / NF, col = j % NF;
      const int f = row / NFF, v = (row % NFF) / NP, mm = row % NP;
      const int f2 = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP;
      const T val = (f == f2) ? ((f < 2) ? wlx : wly) * fs(sh.TLL, f, mm, m2, 12 + v, 4 + v2) : T(0);
      bp[(size_t)(NU + row) * NC + NU + col] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// batched GEMM on the matrix cores (FP64 or FP32): C[b] (+)= alpha A[b] B[b],
// row-major with leading dimensions; 64x64 output tile per workgroup (4 waves x
// 2x2 tiles of the 16x16x4 MFMA), 32-deep k-blocks staged in LDS with the next
// block prefetched into registers.
// ---------------------------------------------------------------------------
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA per element type: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element r of lane l is D[row(l/16, r)][l%16] (the FP64 and FP32
// instructions order the rows differently).
template <class T> struct Mfma16;
template <> struct Mfma16<double> {
  using V = mf_d4;
  __device__ static V op(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma16<float> {
  using V = mf_f4;
  __device__ static V op(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

template <class T, int TILE>
__global__ void __launch_bounds__(256) gemm_kernel(int batch, int M, int N, int Kd, double alpha, int beta_one,
                                                   const T* __restrict__ A, int lda, long long sA,
                                                   const T* __restrict__ B, int ldb, long long sB,
                                                   T* __restrict__ C, int ldc, long long sC) {
  using MF = Mfma16<T>;
  constexpr int KB = 32;                      // k-block staged in LDS
  constexpr int SUB = TILE / 32;              // 16x16 MFMA tiles per wave and dimension
  static_assert(TILE == 32 || TILE == 64, "tile");
  __shared__ T sa[TILE][KB + 1];
  __shared__ T sb[KB][TILE + 1];
  // XCD-aware numbering: the output tiles of one batch entry share an XCD (and its L2)
  const int tn = (N + TILE - 1) / TILE, ntile = ((M + TILE - 1) / TILE) * tn;
  const int L = blockIdx.x, xcd = L & 7, rr = L >> 3;
  const int t = rr % ntile;
  const long long bz = 8LL * (rr / ntile) + xcd;
  if (bz >= batch) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = (t / tn) * TILE, n0 = (t % tn) * TILE;
  const T* Ab = A + bz * sA;
  const T* Bb = B + bz * sB;
  T* Cb = C + bz * sC;
  const int wr = wv >> 1, wc = wv & 1;
  const int li = lane & 15, lk = lane >> 4;
  typename MF::V acc[SUB][SUB];
#pragma unroll
  for (int i = 0; i < SUB; ++i)
#pragma unroll
    for (int j = 0; j < SUB; ++j) acc[i][j] = typename MF::V{T(0), T(0), T(0), T(0)};
  constexpr int NL = TILE * KB / 256;         // elements of each operand block per thread
  T ra[NL], rb[NL];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int idx = tid + 256 * u;
      const int r = idx / KB, kk = idx % KB;
      const int gm = m0 + r, gk = k0 + kk;
      ra[u] = (gm < M && gk < Kd) ? Ab[(size_t)gm * lda + gk] : T(0);
      const int kb = idx / TILE, cc = idx % TILE;
      const int gk2 = k0 + kb, gn = n0 + cc;
      rb[u] = (gk2 < Kd && gn < N) ? Bb[(size_t)gk2 * ldb + gn] : T(0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < Kd; k0 += KB) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int idx = tid + 256 * u;
      sa[idx / KB][idx % KB] = ra[u];
      sb[idx / TILE][idx % TILE] = rb[u];
    }
    __syncthreads();
    if (k0 + KB < Kd) fetch(k0 + KB);
#pragma unroll
    for (int k4 = 0; k4 < KB / 4; ++k4) {
      const int kk = 4 * k4 + lk;
      T av[SUB], bv[SUB];
#pragma unroll
      for (int i = 0; i < SUB; ++i) {
        av[i] = sa[16 * SUB * wr + 16 * i + li][kk];
        bv[i] = sb[kk][16 * SUB * wc + 16 * i + li];
      }
#pragma unroll
      for (int i = 0; i < SUB; ++i)
#pragma unroll
        for (int j = 0; j < SUB; ++j) acc[i][j] = MF::op(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < SUB; ++ti)
#pragma unroll
    for (int tj = 0; tj < SUB; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SUB * wr + 16 * ti + MF::row(lk, r);
        const int gn = n0 + 16 * SUB * wc + 16 * tj + li;
        if (gm < M && gn < N) {
          T* cp = Cb + (size_t)gm * ldc + gn;
          const T v = T(alpha) * acc[ti][tj][r];
          *cp = beta_one ? (*cp + v) : v;
        }
      }
}

// Whole-matrix variant (FP32): a WM x WN grid of waves each holding a (16 SM) x (16 SN)
// block of the output in registers, so that a workgroup covers a BM x BN part of C.  When
// C fits in one part each operand panel is read once per entry (the tiled kernels read it
// once per output tile); larger C is split into parts, one workgroup each, numbered so
// that the parts of one entry run on the same XCD and share its L2 copy of the panels.
// Every 4-deep k-step of a wave issues SM x SN MFMAs from SM + SN LDS reads.  KB-deep
// k-blocks are staged in LDS with the next block prefetched into registers.
template <int WM, int WN, int SM, int SN, int KB, bool SPLIT>
__global__ void __launch_bounds__(64 * WM * WN) gemm_whole_kernel(int batch, int M, int N, int Kd, double alpha,
                                                                  int beta_one, const float* __restrict__ A, int lda,
                                                                  long long sA, const float* __restrict__ B, int ldb,
                                                                  long long sB, float* __restrict__ C, int ldc,
                                                                  long long sC) {
  using MF = Mfma16<float>;
  constexpr int NT = 64 * WM * WN, BM = 16 * SM * WM, BN = 16 * SN * WN;
  constexpr int PA = 4, PB = 16;              // pads: two-way LDS bank pattern for both operands
  static_assert((BM * KB) % NT == 0 && (KB * BN) % NT == 0 && BN % 32 == 0 && KB % 4 == 0, "block shape");
  __shared__ float sa[BM][KB + PA];
  __shared__ float sb[KB][BN + PB];
  int m0 = 0, n0 = 0;
  long long bz = blockIdx.x;
  if constexpr (SPLIT) {
    const int pn = (N + BN - 1) / BN, np = ((M + BM - 1) / BM) * pn;
    const int L = blockIdx.x, xcd = L & 7, rr = L >> 3, part = rr % np;
    bz = 8LL * (rr / np) + xcd;
    m0 = (part / pn) * BM;
    n0 = (part % pn) * BN;
  }
  if (bz >= batch) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv / WN, wc = wv % WN;
  const int li = lane & 15, lk = lane >> 4;
  const float* Ab = A + bz * sA;
  const float* Bb = B + bz * sB;
  float* Cb = C + bz * sC;
  constexpr int NLA = BM * KB / NT, NLB = KB * BN / NT;
  float ra[NLA], rb[NLB];
  // branch-free loads: 32-bit offsets from the entry's base, lanes outside the matrix
  // read its first element, zeroed when staged (a select right after the load would wait
  // for it and keep the next panel's loads from overlapping the matrix products)
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NLA; ++u) {
      const int idx = tid + NT * u;
      const int r = m0 + idx / KB, gk = k0 + idx % KB;
      const bool ok = r < M && gk < Kd;
      ra[u] = Ab[ok ? r * lda + gk : 0];
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
      const int idx = tid + NT * u;
      const int gk = k0 + idx / BN, cc = n0 + idx % BN;
      const bool ok = gk < Kd && cc < N;
      rb[u] = Bb[ok ? gk * ldb + cc : 0];
    }
  };
  typename MF::V acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = typename MF::V{0.0f, 0.0f, 0.0f, 0.0f};
  fetch(0);
  for (int k0 = 0; k0 < Kd; k0 += KB) {
#pragma unroll
    for (int u = 0; u < NLA; ++u) {
      const int idx = tid + NT * u;
      sa[idx / KB][idx % KB] = (m0 + idx / KB < M && k0 + idx % KB < Kd) ? ra[u] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
      const int idx = tid + NT * u;
      sb[idx / BN][idx % BN] = (k0 + idx / BN < Kd && n0 + idx % BN < N) ? rb[u] : 0.0f;
    }
    __syncthreads();
    if (k0 + KB < Kd) fetch(k0 + KB);
#pragma unroll
    for (int k4 = 0; k4 < KB / 4; ++k4) {
      const int kk = 4 * k4 + lk;
      float av[SM], bv[SN];
#pragma unroll
      for (int i = 0; i < SM; ++i) av[i] = sa[16 * SM * wr + 16 * i + li][kk];
#pragma unroll
      for (int j = 0; j < SN; ++j) bv[j] = sb[kk][16 * SN * wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) acc[i][j] = MF::op(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  // C by rows of tiles: all loads of a row before its stores (a store could alias a later
  // load for all the compiler knows, which would serialise every element)
#pragma unroll
  for (int ti = 0; ti < SM; ++ti) {
    float cv[SN][4];
#pragma unroll
    for (int tj = 0; tj < SN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SM * wr + 16 * ti + MF::row(lk, r);
        const int gn = n0 + 16 * SN * wc + 16 * tj + li;
        const bool ok = gm < M && gn < N;
        const float v = Cb[ok ? gm * ldc + gn : 0];
        cv[tj][r] = (beta_one && ok) ? v : 0.0f;
      }
#pragma unroll
    for (int tj = 0; tj < SN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SM * wr + 16 * ti + MF::row(lk, r);
        const int gn = n0 + 16 * SN * wc + 16 * tj + li;
        if (gm < M && gn < N) Cb[gm * ldc + gn] = cv[tj][r] + float(alpha) * acc[ti][tj][r];
      }
  }
}

// Whole-matrix GEMM in FP32 with the products on the bf16 matrix cores: every operand
// entry is split into three bf16 parts, a = a0 + a1 + a2 (a0 = bf16(a), a1 = bf16(a - a0),
// a2 = bf16(a - a0 - a1): 24 significant bits, those of FP32), and a b is accumulated in
// FP32 from the six partial products a_i b_j with i + j <= 2 (the dropped ones are below
// FP32 rounding).  A v_mfma_f32_16x16x16bf16_1k does the work of four FP32 16x16x4 MFMAs
// in a quarter of the time of one, so the six take 1.5 FP32-MFMA times per 16-deep
// k-step instead of 4.  Split parts (workgroup numbering, wave tiles, register prefetch of
// the next k-block, C update) as gemm_whole_kernel; the LDS holds the three bf16 planes
// of the A block with k contiguous and of the B block transposed (k contiguous as well),
// so that each lane reads its four k values of a plane with one 8-byte load.  The splits
// are formed two values at a time with the packed FP32 -> bf16 conversion (round to nearest
// even) and stored as one 32-bit word per plane.
typedef short mf_s4 __attribute__((ext_vector_type(4)));

template <int WM, int WN, int SM, int SN, int KB>
__global__ void __launch_bounds__(64 * WM * WN) gemm_bf3_kernel(int batch, int M, int N, int Kd, double alpha,
                                                                int beta_one, const float* __restrict__ A, int lda,
                                                                long long sA, const float* __restrict__ B, int ldb,
                                                                long long sB, float* __restrict__ C, int ldc,
                                                                long long sC) {
  constexpr int NT = 64 * WM * WN, BM = 16 * SM * WM, BN = 16 * SN * WN;
  constexpr int KP = KB + 4;                  // bf16 row pitch (8-byte aligned rows, staggered banks)
  static_assert(KB % 16 == 0, "block shape");
  __shared__ __align__(16) unsigned short sa[3][BM][KP];
  __shared__ __align__(16) unsigned short sb[3][BN][KP];
  const int pn = (N + BN - 1) / BN, np = ((M + BM - 1) / BM) * pn;
  const int L = blockIdx.x, xcd = L & 7, rr = L >> 3, part = rr % np;
  const long long bz = 8LL * (rr / np) + xcd;
  const int m0 = (part / pn) * BM, n0 = (part % pn) * BN;
  if (bz >= batch) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv / WN, wc = wv % WN;
  const int li = lane & 15, lk = lane >> 4;
  const float* Ab = A + bz * sA;
  const float* Bb = B + bz * sB;
  float* Cb = C + bz * sC;
  // each thread stages pairs of consecutive k values (one packed conversion, one 32-bit
  // LDS store per bf16 plane).  Entries outside the matrices are loaded from a clamped
  // address and zeroed when staged, not when loaded: a select right after a load waits
  // for it, which would keep the next panel's loads from overlapping the matrix products.
  constexpr int PA = BM * KB / 2, PBN = BN * KB / 2;
  constexpr int NLA = (PA + NT - 1) / NT, NLB = (PBN + NT - 1) / NT;
  float ra[NLA][2], rb[NLB][2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NLA; ++u) {
      const int idx = tid + NT * u;
      const int r = m0 + idx / (KB / 2), gk = k0 + 2 * (idx % (KB / 2));
      const bool in = idx < PA && r < M;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool ok = in && gk + e < Kd;
        ra[u][e] = Ab[ok ? r * lda + gk + e : 0];
      }
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
      const int idx = tid + NT * u;
      const int gk = k0 + 2 * (idx / BN), cc = n0 + idx % BN;
      const bool in = idx < PBN && cc < N;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool ok = in && gk + e < Kd;
        rb[u][e] = Bb[ok ? (gk + e) * ldb + cc : 0];
      }
    }
  };
  // x = h0 + h1 + h2 for a pair of values, each part a packed pair of bf16 (round to nearest)
  auto split_pair = [](float x0, float x1, unsigned int (&w)[3]) {
    typedef float vf2 __attribute__((ext_vector_type(2)));
    typedef __bf16 vb2 __attribute__((ext_vector_type(2)));
    float y0 = x0, y1 = x1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const unsigned int h = __builtin_bit_cast(unsigned int, __builtin_convertvector(vf2{y0, y1}, vb2));
      w[q] = h;
      y0 -= __uint_as_float(h << 16);
      y1 -= __uint_as_float(h & 0xffff0000u);
    }
  };
  mf_f4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = mf_f4{0.0f, 0.0f, 0.0f, 0.0f};
  fetch(0);
  for (int k0 = 0; k0 < Kd; k0 += KB) {
#pragma unroll
    for (int u = 0; u < NLA; ++u) {
      const int idx = tid + NT * u;
      if (idx < PA) {
        const int r = idx / (KB / 2), kk = 2 * (idx % (KB / 2));
        const bool rin = m0 + r < M;
        unsigned int w[3];
        split_pair(rin && k0 + kk < Kd ? ra[u][0] : 0.0f, rin && k0 + kk + 1 < Kd ? ra[u][1] : 0.0f, w);
#pragma unroll
        for (int q = 0; q < 3; ++q) *reinterpret_cast<unsigned int*>(&sa[q][r][kk]) = w[q];
      }
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
      const int idx = tid + NT * u;
      if (idx < PBN) {
        const int kk = 2 * (idx / BN), cc = idx % BN;
        const bool cin = n0 + cc < N;
        unsigned int w[3];
        split_pair(cin && k0 + kk < Kd ? rb[u][0] : 0.0f, cin && k0 + kk + 1 < Kd ? rb[u][1] : 0.0f, w);
#pragma unroll
        for (int q = 0; q < 3; ++q) *reinterpret_cast<unsigned int*>(&sb[q][cc][kk]) = w[q];
      }
    }
    __syncthreads();
    if (k0 + KB < Kd) fetch(k0 + KB);
#pragma unroll
    for (int k16 = 0; k16 < KB / 16; ++k16) {
      const int kk = 16 * k16 + 4 * lk;
      mf_s4 av[SM][3], bv[SN][3];
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) av[i][q] = *reinterpret_cast<const mf_s4*>(&sa[q][16 * SM * wr + 16 * i + li][kk]);
#pragma unroll
      for (int j = 0; j < SN; ++j)
#pragma unroll
        for (int q = 0; q < 3; ++q) bv[j][q] = *reinterpret_cast<const mf_s4*>(&sb[q][16 * SN * wc + 16 * j + li][kk]);
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          mf_f4 c = acc[i][j];
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i][2], bv[j][0], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i][1], bv[j][1], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i][0], bv[j][2], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i][1], bv[j][0], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i][0], bv[j][1], c, 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i][0], bv[j][0], c, 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // C by rows of tiles: all loads of a row before its stores
#pragma unroll
  for (int ti = 0; ti < SM; ++ti) {
    float cv[SN][4];
#pragma unroll
    for (int tj = 0; tj < SN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SM * wr + 16 * ti + 4 * lk + r;
        const int gn = n0 + 16 * SN * wc + 16 * tj + li;
        const bool ok = gm < M && gn < N;
        const float v = Cb[ok ? gm * ldc + gn : 0];
        cv[tj][r] = (beta_one && ok) ? v : 0.0f;
      }
#pragma unroll
    for (int tj = 0; tj < SN; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SM * wr + 16 * ti + 4 * lk + r;
        const int gn = n0 + 16 * SN * wc + 16 * tj + li;
        if (gm < M && gn < N) Cb[gm * ldc + gn] = cv[tj][r] + float(alpha) * acc[ti][tj][r];
      }
  }
}

// Whole-matrix shapes: code 2001..2008 -> {WM, WN, SM, SN, KB}.  Several waves per SIMD are
// needed to keep the matrix cores fed (one wave holding a 96 x 96 block runs at half the
// speed of sixteen waves holding 48 x 48 blocks), so the shapes trade block size for waves;
// 2007 and 2008 cover 180 x 180 in two and four parts, with two and five workgroups per CU.
struct WholeShape { int wm, wn, sm, sn, kb; bool split; bool bf3 = false; };
__host__ __device__ constexpr WholeShape whole_shape(int code) {
  return code == 2001 ? WholeShape{4, 4, 3, 3, 32, false}     // 192 x 192, 1024 threads
       : code == 2002 ? WholeShape{2, 4, 6, 3, 32, false}     // 192 x 192, 512 threads
       : code == 2003 ? WholeShape{2, 2, 4, 3, 32, false}     // 128 x 96, 256 threads
       : code == 2004 ? WholeShape{4, 2, 2, 3, 32, false}     // 128 x 96, 512 threads
       : code == 2005 ? WholeShape{5, 2, 1, 3, 40, false}     // 80 x 96, 640 threads
       : code == 2006 ? WholeShape{1, 2, 7, 3, 8, false}      // 112 x 96, 128 threads
       : code == 2007 ? WholeShape{2, 4, 3, 3, 16, true}      // parts of 96 x 192, 512 threads
       : code == 2008 ? WholeShape{2, 2, 3, 3, 16, true}      // parts of 96 x 96, 256 threads
       : code == 2009 ? WholeShape{2, 2, 3, 3, 16, true, true}    // 2008 with split-bf16 products
       : code == 2010 ? WholeShape{2, 4, 3, 3, 16, true, true}    // 2007 with split-bf16 products
       : code == 2011 ? WholeShape{4, 2, 2, 3, 16, true, true}    // parts of 128 x 96 (2004's layout), split bf16
                      : WholeShape{0, 0, 0, 0, 0, false};
}
// workgroups per batch entry of a whole-matrix shape (the output split into parts)
static int gemm_whole_parts(int code, int M, int N) {
  const WholeShape w = whole_shape(code);
  const int bm = 16 * w.sm * w.wm, bn = 16 * w.sn * w.wn;
  return ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
}
static bool gemm_whole_fits(int code, int M, int N) {
  const WholeShape w = whole_shape(code);
  return w.wm > 0 && (w.split || (M <= 16 * w.sm * w.wm && N <= 16 * w.sn * w.wn));
}

// C[b] (+)= alpha A[b] B[b] for b < batch (row-major, leading dimensions lda/ldb/ldc,
// batch strides sA/sB/sC in elements); beta_one selects accumulation into C; tile is
// Full-inner-dimension variant (Kd <= 128, FP32): both panels of an output tile are loaded
// into LDS in one round of global loads, together with the C tile when accumulating, and
// the MFMA sweep then runs without further waits on global memory.  The elimination
// GEMMs (inner dimension 5 (k+1)^2 <= 125) are latency-bound in the k-blocked kernel: one
// long wait per tile instead of one per k-block.
template <int TILE>
__global__ void __launch_bounds__(256) gemm_fk_kernel(int batch, int M, int N, int Kd, double alpha, int beta_one,
                                                      const float* __restrict__ A, int lda, long long sA,
                                                      const float* __restrict__ B, int ldb, long long sB,
                                                      float* __restrict__ C, int ldc, long long sC) {
  using MF = Mfma16<float>;
  constexpr int KM = 128, PA = 4, PB = 16;    // pads: two-way LDS bank pattern (the minimum for 64 lanes)
  constexpr int SUB = TILE / 32;
  static_assert(TILE == 32 || TILE == 64, "tile");
  __shared__ float sa[TILE][KM + PA];
  __shared__ float sb[KM][TILE + PB];
  const int tn = (N + TILE - 1) / TILE, ntile = ((M + TILE - 1) / TILE) * tn;
  const int L = blockIdx.x, xcd = L & 7, rr = L >> 3;
  const int t = rr % ntile;
  const long long bz = 8LL * (rr / ntile) + xcd;
  if (bz >= batch) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = (t / tn) * TILE, n0 = (t % tn) * TILE;
  const float* Ab = A + bz * sA;
  const float* Bb = B + bz * sB;
  float* Cb = C + bz * sC;
  const int wr = wv >> 1, wc = wv & 1;
  const int li = lane & 15, lk = lane >> 4;
  // C tile first (its loads overlap the panel loads)
  float cin[SUB][SUB][4];
#pragma unroll
  for (int ti = 0; ti < SUB; ++ti)
#pragma unroll
    for (int tj = 0; tj < SUB; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SUB * wr + 16 * ti + MF::row(lk, r);
        const int gn = n0 + 16 * SUB * wc + 16 * tj + li;
        cin[ti][tj][r] = (beta_one && gm < M && gn < N) ? Cb[(size_t)gm * ldc + gn] : 0.0f;
      }
  constexpr int NL = TILE * KM / 256;
  float ra[NL], rb[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int idx = tid + 256 * u;
    const int r = idx / KM, kk = idx % KM;
    const int gm = m0 + r;
    ra[u] = (gm < M && kk < Kd) ? Ab[(size_t)gm * lda + kk] : 0.0f;
    const int kb = idx / TILE, cc = idx % TILE;
    const int gn = n0 + cc;
    rb[u] = (kb < Kd && gn < N) ? Bb[(size_t)kb * ldb + gn] : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int idx = tid + 256 * u;
    sa[idx / KM][idx % KM] = ra[u];
    sb[idx / TILE][idx % TILE] = rb[u];
  }
  __syncthreads();
  typename MF::V acc[SUB][SUB];
#pragma unroll
  for (int i = 0; i < SUB; ++i)
#pragma unroll
    for (int j = 0; j < SUB; ++j) acc[i][j] = typename MF::V{0.0f, 0.0f, 0.0f, 0.0f};
  const int nk4 = (Kd + 3) / 4;
  for (int k4 = 0; k4 < nk4; ++k4) {
    const int kk = 4 * k4 + lk;
    float av[SUB], bv[SUB];
#pragma unroll
    for (int i = 0; i < SUB; ++i) {
      av[i] = sa[16 * SUB * wr + 16 * i + li][kk];
      bv[i] = sb[kk][16 * SUB * wc + 16 * i + li];
    }
#pragma unroll
    for (int i = 0; i < SUB; ++i)
#pragma unroll
      for (int j = 0; j < SUB; ++j) acc[i][j] = MF::op(av[i], bv[j], acc[i][j]);
  }
#pragma unroll
  for (int ti = 0; ti < SUB; ++ti)
#pragma unroll
    for (int tj = 0; tj < SUB; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + 16 * SUB * wr + 16 * ti + MF::row(lk, r);
        const int gn = n0 + 16 * SUB * wc + 16 * tj + li;
        if (gm < M && gn < N) Cb[(size_t)gm * ldc + gn] = cin[ti][tj][r] + float(alpha) * acc[ti][tj][r];
      }
}

// the output tile edge (64, or 32 for small matrices; 0 = 64); 1000 + edge selects the
// full-inner-dimension variant (FP32, inner dimension <= 128; otherwise the edge alone);
// 2001..2008 the whole-matrix shapes (FP32; 2001..2006 when the matrix fits one part,
// otherwise edge 64).
template <class T>
static hipError_t gemm_batched(hipStream_t st, int batch, int M, int N, int K, double alpha, bool beta_one,
                               const T* A, int lda, long long sA, const T* B, int ldb, long long sB, T* C, int ldc,
                               long long sC, int tile = 64) {
  if (batch == 0 || M == 0 || N == 0) return hipSuccess;
  if constexpr (std::is_same<T, float>::value) {
    if (tile > 2000 && gemm_whole_fits(tile, M, N)) {
#define WHOLE_LAUNCH(CODE)                                                                                     \
  if (tile == CODE) {                                                                                          \
    constexpr WholeShape ws = whole_shape(CODE);                                                               \
    const long long nbw = 8LL * ((batch + 7) / 8) * gemm_whole_parts(CODE, M, N);                               \
    hipLaunchKernelGGL((gemm_whole_kernel<ws.wm, ws.wn, ws.sm, ws.sn, ws.kb, ws.split>), dim3((unsigned)nbw), \
                       dim3(64 * ws.wm * ws.wn), 0, st, batch, M, N, K, alpha, beta_one ? 1 : 0, A, lda, sA, B, \
                       ldb, sB, C, ldc, sC);                                                                   \
    return hipGetLastError();                                                                                  \
  }
      WHOLE_LAUNCH(2001)
      WHOLE_LAUNCH(2002)
      WHOLE_LAUNCH(2003)
      WHOLE_LAUNCH(2004)
      WHOLE_LAUNCH(2005)
      WHOLE_LAUNCH(2006)
      WHOLE_LAUNCH(2007)
      WHOLE_LAUNCH(2008)
#undef WHOLE_LAUNCH
#define BF3_LAUNCH(CODE)                                                                                       \
  if (tile == CODE) {                                                                                          \
    constexpr WholeShape ws = whole_shape(CODE);                                                               \
    const long long nbw = 8LL * ((batch + 7) / 8) * gemm_whole_parts(CODE, M, N);                               \
    hipLaunchKernelGGL((gemm_bf3_kernel<ws.wm, ws.wn, ws.sm, ws.sn, ws.kb>), dim3((unsigned)nbw),              \
                       dim3(64 * ws.wm * ws.wn), 0, st, batch, M, N, K, alpha, beta_one ? 1 : 0, A, lda, sA, B, \
                       ldb, sB, C, ldc, sC);                                                                   \
    return hipGetLastError();                                                                                  \
  }
      BF3_LAUNCH(2009)
      BF3_LAUNCH(2010)
      BF3_LAUNCH(2011)
#undef BF3_LAUNCH
    }
    if (tile > 1000 && tile < 2000 && K <= 128) {
      const int tf = tile == 1032 ? 32 : 64;
      const long long ntf = (long long)((M + tf - 1) / tf) * ((N + tf - 1) / tf);
      const long long nbf = 8LL * ((batch + 7) / 8) * ntf;
      if (tf == 32)
        hipLaunchKernelGGL((gemm_fk_kernel<32>), dim3((unsigned)nbf), dim3(256), 0, st, batch, M, N, K, alpha,
                           beta_one ? 1 : 0, A, lda, sA, B, ldb, sB, C, ldc, sC);
      else
        hipLaunchKernelGGL((gemm_fk_kernel<64>), dim3((unsigned)nbf), dim3(256), 0, st, batch, M, N, K, alpha,
                           beta_one ? 1 : 0, A, lda, sA, B, ldb, sB, C, ldc, sC);
      return hipGetLastError();
    }
  }
  if (tile > 1000 && tile < 2000) tile -= 1000;
  const int tl = tile == 32 ? 32 : 64;
  const long long nt = (long long)((M + tl - 1) / tl) * ((N + tl - 1) / tl);
  const long long nblk = 8LL * ((batch + 7) / 8) * nt;
  if (tl == 32)
    hipLaunchKernelGGL((gemm_kernel<T, 32>), dim3((unsigned)nblk), dim3(256), 0, st, batch, M, N, K, alpha,
                       beta_one ? 1 : 0, A, lda, sA, B, ldb, sB, C, ldc, sC);
  else
    hipLaunchKernelGGL((gemm_kernel<T, 64>), dim3((unsigned)nblk), dim3(256), 0, st, batch, M, N, K, alpha,
                       beta_one ? 1 : 0, A, lda, sA, B, ldb, sB, C, ldc, sC);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// condensation step 1: K^-1 by in-place Gauss-Jordan with partial pivoting in LDS
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Gauss-Jordan inversion held in registers.  The N x N matrix is spread over
// the workgroup in RT x CT tiles: thread t < (N/RT)(N/CT) owns rows
// (t / (N/CT)) RT .. +RT-1 and columns (t % (N/CT)) CT .. +CT-1.  Partial
// pivoting without row exchanges: step k takes the unused row with the largest
// |A[r][k]| (lowest index on ties), found by every wave on its own from the
// pivot column in LDS; only that column and the pivot row pass through LDS
// (double-buffered, two barriers per step).  On return the tiles hold B with
// A^-1[pos[i]][rp[c]] = B[i][c], where rp[k] is the pivot row of step k and
// pos its inverse (both in LDS).  N <= 128.
// ---------------------------------------------------------------------------
template <int N> struct GJTile;
template <> struct GJTile<8> { static constexpr int RT = 2, CT = 2; };
template <> struct GJTile<12> { static constexpr int RT = 3, CT = 3; };
template <> struct GJTile<16> { static constexpr int RT = 2, CT = 2; };
template <> struct GJTile<20> { static constexpr int RT = 5, CT = 2; };
template <> struct GJTile<36> { static constexpr int RT = 3, CT = 3; };
template <> struct GJTile<40> { static constexpr int RT = 5, CT = 2; };
template <> struct GJTile<60> { static constexpr int RT = 6, CT = 3; };
template <> struct GJTile<64> { static constexpr int RT = 8, CT = 2; };
template <> struct GJTile<80> { static constexpr int RT = 10, CT = 4; };
template <> struct GJTile<100> { static constexpr int RT = 10, CT = 4; };

template <class T> __device__ __forceinline__ T tabs(T x) { return x < T(0) ? -x : x; }
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

}  // namespace imex
// wave-wide maximum from the device library (not declared by every HIP header configuration)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);
namespace imex {

// Pivot keys: the high 32 bits of |a| (monotonic in |a|; sign cleared so -0 ranks as 0)
// above the inverted row index, so one 64-bit wave maximum gives the largest |a| and,
// on ties, the lowest row.
__device__ __forceinline__ unsigned int pivot_bits(float a) { return __float_as_uint(a) & 0x7fffffffu; }
__device__ __forceinline__ unsigned int pivot_bits(double a) {
  return (unsigned int)((unsigned long long)__double_as_longlong(a) >> 32) & 0x7fffffffu;
}
template <class T> __device__ __forceinline__ unsigned long long pivot_key(T a, int row) {
  return ((unsigned long long)pivot_bits(a) << 32) | (unsigned long long)(0xffffffffu - (unsigned int)row);
}

template <int N, class T> struct GJShared {
  T col[2][N];
  T row[2][N];
  int rp[N];
  int pos[N];
};

template <int N, class T>
struct GJ {
  static constexpr int RT = GJTile<N>::RT, CT = GJTile<N>::CT, NCG = N / CT, NTH = (N / RT) * NCG;
  static_assert(N % RT == 0 && N % CT == 0 && NTH <= 256 && N <= 128, "tile shape");
  __device__ static bool owns(int tid) { return tid < NTH; }
  __device__ static int row0(int tid) { return (tid / NCG) * RT; }
  __device__ static int col0(int tid) { return (tid % NCG) * CT; }

  // Tiles start at multiples of RT and CT, so column k sits at register column k % CT of
  // the threads whose tile column starts at k - k % CT, and the pivot row r at register row
  // r % RT of those whose tile row starts at r - r % RT.  Both register indices are the
  // same for every thread (k is the loop counter, r a wave maximum), so with USEL the
  // selection of the register column or row is a scalar branch rather than a per-lane
  // compare and exec-mask branch for every register.  It pays on the 10 x 4 tiles of
  // N >= 80 (k = 4: 559 -> 518 us per inversion of the 4096 K blocks); on the smaller
  // tiles the per-lane form is faster (the compiler keeps the uniform form of the 2 x 2
  // tiles in scratch).
  static constexpr bool USEL = N >= 80;
  __device__ static void invert(T (&A)[RT][CT], GJShared<N, T>& sh, int tid) {
    const bool own = owns(tid);
    const int r0 = row0(tid), c0 = col0(tid);
    const int lane = tid & 63;
    bool used0 = lane >= N, used1 = lane + 64 >= N;
    for (int k = 0; k < N; ++k) {
      T* ck = sh.col[k & 1];
      T* rk = sh.row[k & 1];
      const int jk = k % CT;
      const bool kcol = own && c0 == k - jk;               // this thread holds column k
      if (USEL ? kcol : own) {
#pragma unroll
        for (int j = 0; j < CT; ++j)
          if (USEL ? j == jk : c0 + j == k) {
#pragma unroll
            for (int i = 0; i < RT; ++i) ck[r0 + i] = A[i][j];
          }
      }
      __syncthreads();
      unsigned long long key = used0 ? 0ull : pivot_key(ck[lane], lane);
      if (!used1) {
        const unsigned long long k1 = pivot_key(ck[lane + 64], lane + 64);
        key = k1 > key ? k1 : key;
      }
      key = __ockl_wfred_max_u64(key);
      const int rw = (int)(0xffffffffu - (unsigned int)(key & 0xffffffffull));
      const int r = USEL ? __builtin_amdgcn_readfirstlane(rw) : rw;
      if (r == lane) used0 = true;
      if (r == lane + 64) used1 = true;
      if (tid == 0) { sh.rp[k] = r; sh.pos[r] = k; }
      const int ir = r % RT;
      const bool rrow = USEL ? own && r0 == r - ir : own && r >= r0 && r < r0 + RT;   // holds pivot row r
      if (rrow) {
#pragma unroll
        for (int i = 0; i < RT; ++i)
          if (USEL ? i == ir : r0 + i == r) {
#pragma unroll
            for (int j = 0; j < CT; ++j) rk[c0 + j] = A[i][j];
          }
      }
      __syncthreads();
      const T inv = T(1) / ck[r];
      if (own) {
        T rn[CT], f[RT];
#pragma unroll
        for (int j = 0; j < CT; ++j) rn[j] = rk[c0 + j] * inv;
#pragma unroll
        for (int i = 0; i < RT; ++i) f[i] = ck[r0 + i];
        // rank-1 update everywhere, then the pivot column (-f_i / p) and the
        // normalised pivot row (with 1 / p in the pivot column) overwritten
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j) A[i][j] = tfma(-f[i], rn[j], A[i][j]);
        if (USEL ? kcol : k >= c0 && k < c0 + CT) {
#pragma unroll
          for (int j = 0; j < CT; ++j)
            if (USEL ? j == jk : c0 + j == k) {
#pragma unroll
              for (int i = 0; i < RT; ++i) A[i][j] = -f[i] * inv;
            }
        }
        if (USEL ? rrow : r >= r0 && r < r0 + RT) {
#pragma unroll
          for (int i = 0; i < RT; ++i)
            if (USEL ? i == ir : r0 + i == r) {
#pragma unroll
              for (int j = 0; j < CT; ++j) A[i][j] = (USEL ? kcol && j == jk : c0 + j == k) ? inv : rn[j];
            }
        }
      }
    }
    __syncthreads();
  }
};

template <int K, class T>
__global__ void __launch_bounds__(256) hdg_invert_kernel(size_t blk_stride, const T* __restrict__ blk,
                                                         T* __restrict__ Kinv) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NC = NU + NF + 1;
  using G = GJ<NU, T>;
  __shared__ GJShared<NU, T> sh;
  const int p = blockIdx.x, tid = threadIdx.x;
  const T* bp = blk + (size_t)p * blk_stride;
  const int r0 = G::row0(tid), c0 = G::col0(tid);
  const bool own = G::owns(tid);
  T A[G::RT][G::CT];
#pragma unroll
  for (int i = 0; i < G::RT; ++i)
#pragma unroll
    for (int j = 0; j < G::CT; ++j) A[i][j] = own ? bp[(size_t)(r0 + i) * NC + c0 + j] : T(0);
  G::invert(A, sh, tid);
  if (!own) return;
  T* Kp = Kinv + (size_t)p * NU * NU;
#pragma unroll
  for (int i = 0; i < G::RT; ++i) {
    const int row = sh.pos[r0 + i];
#pragma unroll
    for (int j = 0; j < G::CT; ++j) Kp[(size_t)row * NU + sh.rp[c0 + j]] = A[i][j];
  }
}

// ---------------------------------------------------------------------------
// K^-1 in FP32 by blocked in-place Gauss-Jordan on the matrix cores.  The NU x NU block
// sits column-major in LDS (columns padded to whole 16 x 16 tiles with zeros).  Pivots go
// in panels of 16: the wave that owns a panel's tile column factorises the panel in
// registers (each lane holds rows lane, lane + 64 of the 16 columns; partial pivoting
// among the rows not yet used, by a wave-wide maximum of |a|, lowest row on ties), which
// gives the panel transformation's columns T[:, r_t] for its pivot rows r_t.  Every other
// column then takes the rank-16 update A[:, j] += (T[:, r] - I[:, r]) A[r, j] on
// v_mfma_f32_16x16x4f32 tiles (accumulators loaded from and stored back to LDS), and the
// panel's own columns become T[:, r].  In-place Gauss-Jordan keeps the accumulated
// transformation in the pivoted columns, so after NU pivots the block holds K^-1 with
// rows and columns permuted by the pivot order: K^-1[q][c] = A[rp[q]][pos[c]].
// Column tiles are dealt round robin to the four waves; each wave updates all row tiles
// of its columns, so a panel's pivot-row values are read and written by the same wave.
// ---------------------------------------------------------------------------
// LDS of the blocked Gauss-Jordan on an N x N matrix: the matrix column-major with its
// columns padded to whole 16 x 16 tiles (TN floats per column, zeros beyond N), the
// transformation buffer [PB][TN], and the pivot tables rp, pos (N ints each).
template <int N> struct GjbDims {
  static constexpr int TT = (N + 15) / 16, TN = 16 * TT;             // tiles per side, padded size
  static constexpr int PB = 16, RPL = (N + 63) / 64;                 // pivots per panel, rows per lane
  static_assert(N % 4 == 0, "float4 column segments");
  static constexpr size_t FLOATS = (size_t)TN * N + (size_t)PB * TN, INTS = 2 * (size_t)N;
  static constexpr size_t BYTES = sizeof(float) * FLOATS + sizeof(int) * INTS;
};

// In-place inverse of the N x N matrix Am (column j at Am + j * N, columns N..TN-1 zero)
// by the 256 threads of the workgroup; on entry Tb is zero and pos[] = -1, and the caller
// has synchronised.  On return (synchronised) A^-1[q][c] = Am[pos[c] * N + rp[q]].
template <int N>
__device__ __forceinline__ void gj_blocked(float* __restrict__ Am, float* __restrict__ Tb, int* __restrict__ rp,
                           int* __restrict__ pos, int tid) {
  using D = GjbDims<N>;
  constexpr int TT = D::TT, TN = D::TN, PB = D::PB, RPL = D::RPL;
  constexpr int TPW = (TT + 3) / 4;                      // tile columns per wave
  const int lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int p0 = 0; p0 < N; p0 += PB) {
    const int nb = N - p0 < PB ? N - p0 : PB;
    const int owner = (p0 / 16) & 3;                     // the wave holding the panel's tile column
    float P[RPL][PB];
    int rpan[PB];
    if (wv == owner) {
      bool avail[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int row = lane + 64 * s;
        avail[s] = row < N && pos[row < N ? row : 0] < 0;
#pragma unroll
        for (int cc = 0; cc < PB; ++cc) P[s][cc] = (row < N && cc < nb) ? Am[(p0 + cc) * N + row] : 0.0f;
      }
#pragma unroll
      for (int t = 0; t < PB; ++t) {
        rpan[t] = 0;
        if (t < nb) {
          unsigned long long key = 0ull;
#pragma unroll
          for (int s = 0; s < RPL; ++s)
            if (avail[s]) {
              const unsigned long long kk = pivot_key(P[s][t], lane + 64 * s);
              key = kk > key ? kk : key;
            }
          key = __ockl_wfred_max_u64(key);
          const int r = (int)(0xffffffffu - (unsigned int)(key & 0xffffffffull));
          rpan[t] = r;
          const int sr = r >> 6, lr = r & 63;
          float prow[PB];
#pragma unroll
          for (int cc = 0; cc < PB; ++cc) {
            float v = P[0][cc];
#pragma unroll
            for (int s = 1; s < RPL; ++s) v = (sr == s) ? P[s][cc] : v;
            prow[cc] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lr));
          }
          const float inv = 1.0f / prow[t];
#pragma unroll
          for (int cc = 0; cc < PB; ++cc) prow[cc] *= inv;
#pragma unroll
          for (int s = 0; s < RPL; ++s) {
            const bool me = (lane + 64 * s) == r;
            const float m = P[s][t];
#pragma unroll
            for (int cc = 0; cc < PB; ++cc) {
              const float up = me ? prow[cc] : __builtin_fmaf(-m, prow[cc], P[s][cc]);
              P[s][cc] = (cc == t) ? (me ? inv : -m * inv) : up;
            }
            if (me) avail[s] = false;
          }
        }
      }
    }
    __syncthreads();                                     // every wave is done with the last panel's T
    if (wv == owner) {
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int row = lane + 64 * s;
        if (row < N) {
#pragma unroll
          for (int cc = 0; cc < PB; ++cc)
            Tb[cc * TN + row] = (cc < nb) ? P[s][cc] - (row == rpan[cc] ? 1.0f : 0.0f) : 0.0f;
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int t = 0; t < PB; ++t)
          if (t < nb) { rp[p0 + t] = rpan[t]; pos[rpan[t]] = p0 + t; }
      }
    }
    __syncthreads();
    // rank-nb update of this wave's tile columns; the pivot-row values of its columns are
    // read before any of its tiles is written
    float bvs[TPW][PB / 4];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int col = 16 * (wv + 4 * q) + li;
#pragma unroll
      for (int ks = 0; ks < PB / 4; ++ks) {
        const int t = 4 * ks + lk;
        bvs[q][ks] = (t < nb && wv + 4 * q < TT) ? Am[col * N + rp[p0 + (t < nb ? t : 0)]] : 0.0f;
      }
    }
#pragma unroll
    for (int qc = 0; qc < TPW; ++qc) {
      const int tj = wv + 4 * qc;
      if (tj >= TT) break;
      const int col = 16 * tj + li;
      const bool pcol = col >= p0 && col < p0 + nb;
      const int tp = pcol ? col - p0 : 0;
      const int prow_t = rp[p0 + tp];
#pragma unroll
      for (int ti = 0; ti < TT; ++ti) {
        const int r0 = 16 * ti + 4 * lk;
        const bool rows_ok = r0 < N;
        mf_f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        if (rows_ok) {
          const float4 cv = *reinterpret_cast<const float4*>(Am + col * N + r0);
          acc = mf_f4{cv.x, cv.y, cv.z, cv.w};
        }
#pragma unroll
        for (int ks = 0; ks < PB / 4; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Tb[(4 * ks + lk) * TN + 16 * ti + li], bvs[qc][ks], acc, 0, 0, 0);
        if (rows_ok) {
          float4 o = make_float4(acc[0], acc[1], acc[2], acc[3]);
          if (pcol) {
            const float* tc = Tb + tp * TN + r0;
            o = make_float4(tc[0] + (r0 == prow_t ? 1.0f : 0.0f), tc[1] + (r0 + 1 == prow_t ? 1.0f : 0.0f),
                            tc[2] + (r0 + 2 == prow_t ? 1.0f : 0.0f), tc[3] + (r0 + 3 == prow_t ? 1.0f : 0.0f));
          }
          *reinterpret_cast<float4*>(Am + col * N + r0) = o;
        }
      }
    }
  }
  __syncthreads();
}

template <int K> struct GjiDims {
  static constexpr int NU = 4 * (K + 1) * (K + 1);
  static constexpr size_t LDS = GjbDims<NU>::BYTES;
};

template <int K>
__global__ void __launch_bounds__(256) hdg_invert_mfma_kernel(size_t bs, const float* __restrict__ blk,
                                                              float* __restrict__ Kinv) {
  using D = GjbDims<GjiDims<K>::NU>;
  constexpr int NU = GjiDims<K>::NU, TN = D::TN, PB = D::PB;
  constexpr int NC = NU + 16 * (K + 1) + 1;              // row stride of the element block
  extern __shared__ __align__(16) float gji_lds[];
  float* Am = gji_lds;                                   // column j at Am + j * NU
  float* Tb = Am + (size_t)TN * NU;                      // [PB][TN]: T[:, r_t] - e_{r_t}
  int* rp = reinterpret_cast<int*>(Tb + PB * TN);        // [NU] pivot row of pivot k
  int* pos = rp + NU;                                    // [NU] pivot index of row r (-1: not yet)
  const int tid = threadIdx.x;
  const float* bp = blk + (size_t)blockIdx.x * bs;
  for (int idx = tid; idx < NU * NU; idx += 256) {
    const int r = idx / NU, cc = idx - r * NU;
    Am[cc * NU + r] = bp[(size_t)r * NC + cc];
  }
  for (int idx = tid; idx < (TN - NU) * NU; idx += 256) Am[NU * NU + idx] = 0.0f;
  for (int idx = tid; idx < PB * TN; idx += 256) Tb[idx] = 0.0f;
  for (int idx = tid; idx < NU; idx += 256) pos[idx] = -1;
  __syncthreads();
  gj_blocked<NU>(Am, Tb, rp, pos, tid);
  float* Kp = Kinv + (size_t)blockIdx.x * NU * NU;
  for (int idx = tid; idx < NU * NU; idx += 256) {
    const int q = idx / NU, cc = idx - q * NU;
    Kp[idx] = Am[pos[cc] * NU + rp[q]];
  }
}

// ---------------------------------------------------------------------------
// facet system
// ---------------------------------------------------------------------------
// b_F = sum_T -(h_T - D_T K_T^-1 f_T)|_F: h_T (FP64) plus the last column of the condensed
// augmented system, which holds -D_T K_T^-1 f_T
template <int K, class T>
__global__ void facet_rhs_kernel(DeviceHDG h, size_t blk_stride, const T* __restrict__ blk,
                                 const double* __restrict__ hres, double* __restrict__ b) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * NFF) return;
  const int hf = t / NFF, row = t % NFF;
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * hf + s];
    if (pe < 0) continue;
    const int f = h.hf_face[2 * hf + s];
    const int lr = f * NFF + row;
    acc -= hres[(size_t)pe * NF + lr] + (double)blk[(size_t)pe * blk_stride + (size_t)(NU + lr) * NC + NC - 1];
  }
  b[t] = acc;
}

// ---------------------------------------------------------------------------
// facet preconditioner: restricted additive Schwarz on two-column windows.
// Each window's restriction of S is block-tridiagonal over its super-rows
// (element rows; 5 facet slots each).  The factorisation keeps explicit inverses
// of the eliminated diagonal blocks so that the apply is a chain of GEMVs.
// Global storage is column-major (transposed) for coalesced GEMVs.
// ---------------------------------------------------------------------------
// S[F, G] for HDG facets F, G (NFF x NFF block entry (i, j)): sum over the
// implicit elements having both as faces of their condensed blocks S_T.
// Offsets (into the condensed element systems) of the S_T blocks that couple
// facet F (rows) to facet G (columns): for each side of F the element's facet
// block of face G (up to two faces, for one-element periodic strips); -1 if none.
template <int K>
__device__ void s_block_offsets(const DeviceHDG& h, size_t bs, int F, int G, long long off[4]) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  off[0] = off[1] = off[2] = off[3] = -1;
  if (F < 0 || G < 0) return;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * F + s];
    if (pe < 0) continue;
    const int lf = h.hf_face[2 * F + s];
    int nm = 0;
    for (int lg = 0; lg < 4 && nm < 2; ++lg)
      if (h.efacet[4 * pe + lg] == G)
        off[2 * s + nm++] = (long long)pe * (long long)bs + (long long)(NU + lf * NFF) * NC + NU + lg * NFF;
  }
}

// Branch-free: a missing share (offset -1) reads S[0] and takes zero, so that a thread's
// gathers are issued together instead of one conditional load (and its wait) at a time.
template <class T>
__device__ __forceinline__ T s_gather(const T* __restrict__ S, const long long* off, int i, int j, int ld) {
  T v = T(0);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bool ok = off[t] >= 0;
    const T x = S[ok ? off[t] + (long long)i * ld + j : 0];
    v += ok ? x : T(0);
  }
  return v;
}

// Factorisation of the restricted additive Schwarz windows: each window is a
// chain of super-rows (5 facet slots, NB unknowns) coupled block-tridiagonally
// through the horizontal slots (first NH unknowns).  Forward block elimination
// with explicit inverses: D_r = A_r - B_r D_{r-1}^-1 C_{r-1} on the NH x NH
// corner, G_r = B_r D_{r-1}^-1.  The diagonal block lives in register tiles
// (GJ<NB>), the previous inverse, B_r / G_r and C_{r-1} in LDS; it is inverted by the
// register Gauss-Jordan in FP64 and by the blocked one (gj_blocked) in FP32.  Stored for the
// apply: D_r^-1, G_r and E_r = D_r^-1 C_r, each transposed for coalesced
// matrix-vector products.
template <int K, class T>
__global__ void __launch_bounds__(256) ras_factor_kernel(DeviceHDG h, const T* __restrict__ S, size_t bs,
                                                         T* __restrict__ Wd, T* __restrict__ Wg,
                                                         T* __restrict__ Wc) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NB = 5 * NFF, NH = 2 * NFF;
  constexpr int NC = NU + NF + 1;
  using G = GJ<NB, T>;
  extern __shared__ __align__(16) unsigned char smem_bytes[];
  T* Ds = reinterpret_cast<T*>(smem_bytes);   // NB x NB: D_{r-1}^-1 (row-major)
  T* Bs = Ds + NB * NB;                       // NH x NB: B_r, then G_r
  T* Cs = Bs + NH * NB;                       // NB x NH: C_{r-1}
  T* Us = Cs + NB * NH;                       // NH x NH: G_r C_{r-1}
  __shared__ GJShared<NB, T> gsh;
  __shared__ int fs[5], fp[5];
  __shared__ long long oA[5][5][4], oB[2][5][4], oC[5][2][4];
  const int w = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int g0 = h.win_off[w], g1 = h.win_off[w + 1];
  const bool own = G::owns(tid);
  const int r0 = G::row0(tid), c0 = G::col0(tid);
  // G_r = B_r D^-1 is NH x NB: 4 x 4 register tiles over (NH/4) x (NB/4) threads
  constexpr int GR = 4, GC = 4, NGC = NB / GC, NGT = (NH / GR) * NGC;
  static_assert(NH % GR == 0 && NB % GC == 0 && NGT <= 256, "G tile shape");
  // E_{r-1} = D_{r-1}^-1 C_{r-1} is NB x NH: 4 x 4 tiles
  constexpr int ER = 4, EC = 4, NEC = NH / EC, NET = (NB / ER) * NEC;
  static_assert(NB % ER == 0 && NH % EC == 0 && NET <= 256, "E tile shape");
  // G_r C_{r-1} is NH x NH: 2 x 4 tiles
  constexpr int UR = 2, UC = 4, NUC = NH / UC, NUT = (NH / UR) * NUC;
  static_assert(NH % UR == 0 && NH % UC == 0 && NUT <= 256, "corner tile shape");
  for (int g = g0; g < g1; ++g) {
    if (tid < 5) {
      fs[tid] = h.win_slot[5 * g + tid];
      fp[tid] = (g > g0) ? h.win_slot[5 * (g - 1) + tid] : -1;
    }
    __syncthreads();
    if (tid < 25) s_block_offsets<K>(h, bs, fs[tid / 5], fs[tid % 5], oA[tid / 5][tid % 5]);
    else if (tid < 35) s_block_offsets<K>(h, bs, fs[(tid - 25) / 5], fp[(tid - 25) % 5], oB[(tid - 25) / 5][(tid - 25) % 5]);
    else if (tid < 45) s_block_offsets<K>(h, bs, fp[(tid - 35) / 2], fs[(tid - 35) % 2], oC[(tid - 35) / 2][(tid - 35) % 2]);
    __syncthreads();
    // the diagonal block (identity rows and columns for empty slots); lanes without a
    // tile gather entry (0, 0) and discard it
    T A[G::RT][G::CT];
#pragma unroll
    for (int i = 0; i < G::RT; ++i)
#pragma unroll
      for (int j = 0; j < G::CT; ++j) {
        const int r = own ? r0 + i : 0, c = own ? c0 + j : 0;
        const int a = r / NFF, b = c / NFF;
        const T v = s_gather(S, oA[a][b], r % NFF, c % NFF, NC);
        A[i][j] = !own ? T(0) : (fs[a] < 0 || fs[b] < 0) ? ((r == c) ? T(1) : T(0)) : v;
      }
    if (g > g0) {
      constexpr int NBC = (NH * NB + 255) / 256;   // entries of B_r (and of C_{r-1}) per thread
      {
        T bv[NBC];
#pragma unroll
        for (int u = 0; u < NBC; ++u) {
          const int idx = tid + 256 * u, q = idx < NH * NB ? idx : 0;
          const int r = q / NB, c = q % NB;
          bv[u] = s_gather(S, oB[r / NFF][c / NFF], r % NFF, c % NFF, NC);
        }
#pragma unroll
        for (int u = 0; u < NBC; ++u)
          if (tid + 256 * u < NH * NB) Bs[tid + 256 * u] = bv[u];
      }
      {
        T cv[NBC];
#pragma unroll
        for (int u = 0; u < NBC; ++u) {
          const int idx = tid + 256 * u, q = idx < NB * NH ? idx : 0;
          const int r = q / NH, c = q % NH;
          cv[u] = s_gather(S, oC[r / NFF][c / NFF], r % NFF, c % NFF, NC);
        }
#pragma unroll
        for (int u = 0; u < NBC; ++u)
          if (tid + 256 * u < NB * NH) Cs[tid + 256 * u] = cv[u];
      }
      __syncthreads();
      // G_r = B_r D_{r-1}^-1
      T gt[GR][GC];
#pragma unroll
      for (int i = 0; i < GR; ++i)
#pragma unroll
        for (int j = 0; j < GC; ++j) gt[i][j] = T(0);
      const int gr0 = (tid / NGC) * GR, gc0 = (tid % NGC) * GC;
      if (tid < NGT) {
        for (int k = 0; k < NB; ++k) {
          T bv[GR], dv[GC];
#pragma unroll
          for (int i = 0; i < GR; ++i) bv[i] = Bs[(gr0 + i) * NB + k];
#pragma unroll
          for (int j = 0; j < GC; ++j) dv[j] = Ds[k * NB + gc0 + j];
#pragma unroll
          for (int i = 0; i < GR; ++i)
#pragma unroll
            for (int j = 0; j < GC; ++j) gt[i][j] += bv[i] * dv[j];
        }
      }
      __syncthreads();
      // E_{r-1} = D_{r-1}^-1 C_{r-1} (NB x NH), stored transposed: E[k * NB + i] = E_{r-1}[i][k]
      if (tid < NET) {
        const int er0 = (tid / NEC) * ER, ec0 = (tid % NEC) * EC;
        T et[ER][EC];
#pragma unroll
        for (int i = 0; i < ER; ++i)
#pragma unroll
          for (int j = 0; j < EC; ++j) et[i][j] = T(0);
        for (int k = 0; k < NB; ++k) {
          T dv[ER], cv[EC];
#pragma unroll
          for (int i = 0; i < ER; ++i) dv[i] = Ds[(er0 + i) * NB + k];
#pragma unroll
          for (int j = 0; j < EC; ++j) cv[j] = Cs[k * NH + ec0 + j];
#pragma unroll
          for (int i = 0; i < ER; ++i)
#pragma unroll
            for (int j = 0; j < EC; ++j) et[i][j] += dv[i] * cv[j];
        }
        T* Eg = Wc + (size_t)(g - 1) * NB * NH;
#pragma unroll
        for (int i = 0; i < ER; ++i)
#pragma unroll
          for (int j = 0; j < EC; ++j) Eg[(size_t)(ec0 + j) * NB + er0 + i] = et[i][j];
      }
      if (tid < NGT) {
        T* Gg = Wg + (size_t)g * NH * NB;
#pragma unroll
        for (int i = 0; i < GR; ++i)
#pragma unroll
          for (int j = 0; j < GC; ++j) {
            Bs[(gr0 + i) * NB + gc0 + j] = gt[i][j];
            Gg[(size_t)(gc0 + j) * NH + gr0 + i] = gt[i][j];
          }
      }
      __syncthreads();
      // U = G_r C_{r-1} (NH x NH), then A[H, H] -= U by the tile owners
      if (tid < NUT) {
        const int ur0 = (tid / NUC) * UR, uc0 = (tid % NUC) * UC;
        T ut[UR][UC];
#pragma unroll
        for (int i = 0; i < UR; ++i)
#pragma unroll
          for (int j = 0; j < UC; ++j) ut[i][j] = T(0);
        for (int k = 0; k < NB; ++k) {
          T gv[UR], cv[UC];
#pragma unroll
          for (int i = 0; i < UR; ++i) gv[i] = Bs[(ur0 + i) * NB + k];
#pragma unroll
          for (int j = 0; j < UC; ++j) cv[j] = Cs[k * NH + uc0 + j];
#pragma unroll
          for (int i = 0; i < UR; ++i)
#pragma unroll
            for (int j = 0; j < UC; ++j) ut[i][j] += gv[i] * cv[j];
        }
#pragma unroll
        for (int i = 0; i < UR; ++i)
#pragma unroll
          for (int j = 0; j < UC; ++j) Us[(ur0 + i) * NH + uc0 + j] = ut[i][j];
      }
      __syncthreads();
      if (own && r0 < NH && c0 < NH) {
#pragma unroll
        for (int i = 0; i < G::RT; ++i)
#pragma unroll
          for (int j = 0; j < G::CT; ++j)
            if (r0 + i < NH && c0 + j < NH) A[i][j] -= Us[(r0 + i) * NH + c0 + j];
      }
    }
    T* Dg = Wd + (size_t)g * NB * NB;
    if constexpr (std::is_same<T, float>::value) {
      // FP32: the blocked Gauss-Jordan (pivots of a panel within one wave, rank-16 updates
      // on the matrix cores) on the block column-major in LDS; one window per CU leaves the
      // register Gauss-Jordan waiting on its barriers at every pivot
      using GB = GjbDims<NB>;
      float* Am = Us + NH * NH;
      float* Tb = Am + (size_t)GB::TN * NB;
      int* rpb = reinterpret_cast<int*>(Tb + GB::PB * GB::TN);
      int* posb = rpb + NB;
      if (own) {
#pragma unroll
        for (int i = 0; i < G::RT; ++i)
#pragma unroll
          for (int j = 0; j < G::CT; ++j) Am[(c0 + j) * NB + r0 + i] = A[i][j];
      }
      for (int idx = tid; idx < (GB::TN - NB) * NB; idx += nt) Am[NB * NB + idx] = 0.0f;
      for (int idx = tid; idx < GB::PB * GB::TN; idx += nt) Tb[idx] = 0.0f;
      for (int idx = tid; idx < NB; idx += nt) posb[idx] = -1;
      __syncthreads();
      gj_blocked<NB>(Am, Tb, rpb, posb, tid);
      // D_r^-1[q][c] = Am[pos[c]][rp[q]]: transposed to global (coalesced over q), row-major
      // to LDS for the next super-row
      for (int idx = tid; idx < NB * NB; idx += nt) {
        const int c = idx / NB, q = idx - c * NB;
        const float v = Am[posb[c] * NB + rpb[q]];
        Dg[(size_t)c * NB + q] = v;
        Ds[q * NB + c] = v;
      }
      __syncthreads();
    } else {
      G::invert(A, gsh, tid);
      // D_r^-1: transposed to global, row-major (un-permuted) to LDS for the next super-row
      if (own) {
#pragma unroll
        for (int i = 0; i < G::RT; ++i) {
          const int row = gsh.pos[r0 + i];
#pragma unroll
          for (int j = 0; j < G::CT; ++j) {
            const int col = gsh.rp[c0 + j];
            Dg[(size_t)col * NB + row] = A[i][j];
            Ds[row * NB + col] = A[i][j];
          }
        }
      }
      __syncthreads();
    }
  }
}

// Workgroup barrier for exchanges through LDS only.  __syncthreads() also orders global
// memory, which makes every wave wait for all of its outstanding global loads, prefetches
// included; the k = 4 Schwarz sweep exchanges only LDS values between threads (each thread
// reads back only global values it wrote itself), so its barriers wait for LDS operations
// alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sweep sizes of a super-row of the facet preconditioner's windows: NB unknowns (five
// facet slots), the first NH of them (the two horizontal slots) coupling consecutive
// super-rows; per super-row NSV doubles of Wy, of which the apply keeps w_r at offset NB.
template <int K> struct RasDims {
  static constexpr int NFF = 4 * (K + 1), NB = 5 * NFF, NH = 2 * NFF, NSV = 2 * NB + NH;
};

// Preconditioner apply z = M^-1 x in one launch: one workgroup per window sweeps its
// super-rows forward, y_r = x_r - G_r [y_{r-1}[H]; x_{r-1}[~H]] (only the H rows change)
// and w_r = D_r^-1 y_r (w_r kept in Wy), then backward, z_r = w_r - E_r z_{r+1}[H] with the
// owned facets of z_r written.  Each product is split into column slices over the 256
// threads (partial sums reduced through LDS, FP64 accumulation of the FP32 or FP64
// factors), and the next super-row's factor entries and vector values are loaded into
// registers while the current super-row is applied, so the factor stream, not the serial
// chain, sets the pace.
template <int K, class T>
__global__ void __launch_bounds__(256) ras_apply_kernel(DeviceHDG h, const T* __restrict__ Wg, const T* __restrict__ Wd,
                                                        const T* __restrict__ Wc, const double* __restrict__ x,
                                                        double* __restrict__ Wy, double* __restrict__ z) {
  using D = RasDims<K>;
  constexpr int NFF = D::NFF, NB = D::NB, NH = D::NH;
  constexpr int PD = 256 / NB, CD = (NB + PD - 1) / PD;      // D^-1: NB rows, NB columns
  constexpr int PG = 256 / NH, CG = (NB + PG - 1) / PG;      // G: NH rows, NB columns
  constexpr int PE = 256 / NB, CE = (NH + PE - 1) / PE;      // E: NB rows, NH columns
  __shared__ double yv[NB], prev[NB], zn[NH], pd[PD][NB], pg[PG][NH], pe[PE][NB];
  const int w = blockIdx.x, t = threadIdx.x;
  const int g0 = h.win_off[w], g1 = h.win_off[w + 1];
  if (g1 <= g0) return;
  const int di = t % NB, dq = t / NB;                        // D^-1 and E row / slice of this thread
  const int gi = t % NH, gq = t / NH;                        // G row / slice
  const bool dON = t < PD * NB, gON = t < PG * NH, eON = t < PE * NB;
  auto xval = [&](int g, int i) -> double {
    const int f = h.win_slot[5 * g + i / NFF];
    return f >= 0 ? x[(size_t)f * NFF + i % NFF] : 0.0;
  };
  T gr[CG], dr[CD];
  auto load_fwd = [&](int g) {
    const T* Gg = Wg + (size_t)g * NH * NB;                  // Gg[k * NH + i] = G_r[i][k]
    const T* Dg = Wd + (size_t)g * NB * NB;                  // Dg[k * NB + i] = D_r^-1[i][k]
#pragma unroll
    for (int kk = 0; kk < CG; ++kk) {
      const int k = gq * CG + kk;
      gr[kk] = (gON && g > g0 && k < NB) ? Gg[(size_t)k * NH + gi] : T(0);
    }
#pragma unroll
    for (int kk = 0; kk < CD; ++kk) {
      const int k = dq * CD + kk;
      dr[kk] = (dON && k < NB) ? Dg[(size_t)k * NB + di] : T(0);
    }
  };
  load_fwd(g0);
  double xn = t < NB ? xval(g0, t) : 0.0;
  for (int g = g0; g < g1; ++g) {
    if (t < NB) yv[t] = xn;
    __syncthreads();
    T gc[CG], dc[CD];
#pragma unroll
    for (int kk = 0; kk < CG; ++kk) gc[kk] = gr[kk];
#pragma unroll
    for (int kk = 0; kk < CD; ++kk) dc[kk] = dr[kk];
    if (g + 1 < g1) {
      load_fwd(g + 1);
      xn = t < NB ? xval(g + 1, t) : 0.0;
    }
    if (g > g0) {
      if (gON) {
        double a = 0.0;
#pragma unroll
        for (int kk = 0; kk < CG; ++kk) {
          const int k = gq * CG + kk;
          if (k < NB) a += (double)gc[kk] * prev[k];
        }
        pg[gq][gi] = a;
      }
      __syncthreads();
      if (t < NH) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < PG; ++q) a += pg[q][t];
        yv[t] -= a;
      }
      __syncthreads();
    }
    if (dON) {
      double a = 0.0;
#pragma unroll
      for (int kk = 0; kk < CD; ++kk) {
        const int k = dq * CD + kk;
        if (k < NB) a += (double)dc[kk] * yv[k];
      }
      pd[dq][di] = a;
    }
    if (t < NB) prev[t] = yv[t];
    __syncthreads();
    if (t < NB) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < PD; ++q) a += pd[q][t];
      Wy[(size_t)g * D::NSV + NB + t] = a;                   // w_r, read back by this thread
    }
  }
  // backward sweep
  T er[CE];
  auto load_bwd = [&](int g) {
    const T* Eg = Wc + (size_t)g * NB * NH;                  // Eg[k * NB + i] = E_r[i][k]
#pragma unroll
    for (int kk = 0; kk < CE; ++kk) {
      const int k = dq * CE + kk;
      er[kk] = (eON && k < NH) ? Eg[(size_t)k * NB + di] : T(0);
    }
  };
  if (g1 - 2 >= g0) load_bwd(g1 - 2);
  for (int g = g1 - 1; g >= g0; --g) {
    double v = t < NB ? Wy[(size_t)g * D::NSV + NB + t] : 0.0;
    if (g < g1 - 1) {
      T ec[CE];
#pragma unroll
      for (int kk = 0; kk < CE; ++kk) ec[kk] = er[kk];
      if (g - 1 >= g0) load_bwd(g - 1);
      if (eON) {
        double a = 0.0;
#pragma unroll
        for (int kk = 0; kk < CE; ++kk) {
          const int k = dq * CE + kk;
          if (k < NH) a += (double)ec[kk] * zn[k];
        }
        pe[dq][di] = a;
      }
      __syncthreads();
      if (t < NB) {
#pragma unroll
        for (int q = 0; q < PE; ++q) v -= pe[q][t];
      }
    }
    __syncthreads();                                         // zn and pe free again
    if (t < NB) {
      if (t < NH) zn[t] = v;
      const int a = t / NFF;
      const int f = h.win_slot[5 * g + a];
      if (f >= 0 && h.win_own[5 * g + a]) z[(size_t)f * NFF + t % NFF] = v;
    }
    __syncthreads();
  }
}

// The same apply for k = 4 with 16-byte factor loads: each product is split over the 256
// threads into groups of V consecutive rows (one 16-byte load per column: V = 4 in FP32,
// 2 in FP64) times slices of columns.  A thread's prefetch of the next super-row is then
// about a dozen loads instead of the 67 of one row per thread, which is more than a wave
// can have in flight.  (At lower degrees one row per thread is faster: it needs fewer
// registers and less LDS, so more of an ensemble's many short windows share a CU.)
template <class T> struct Ld16;
template <> struct Ld16<float> {
  static constexpr int V = 4;
  __device__ static void get(const float* p, float (&o)[4]) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
  }
};
template <> struct Ld16<double> {
  static constexpr int V = 2;
  __device__ static void get(const double* p, double (&o)[2]) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    o[0] = q.x; o[1] = q.y;
  }
};

template <int K, class T>
__global__ void __launch_bounds__(256) ras_apply16_kernel(DeviceHDG h, const T* __restrict__ Wg, const T* __restrict__ Wd,
                                                        const T* __restrict__ Wc, const double* __restrict__ x,
                                                        double* __restrict__ Wy, double* __restrict__ z) {
  using D = RasDims<K>;
  using L = Ld16<T>;
  constexpr int NFF = D::NFF, NB = D::NB, NH = D::NH, V = L::V;
  static_assert(NB % V == 0 && NH % V == 0, "row groups");
  constexpr int RD = NB / V, SD = 256 / RD, CD = (NB + SD - 1) / SD;   // D^-1: NB rows, NB columns
  constexpr int RG = NH / V, SG = 256 / RG, CG = (NB + SG - 1) / SG;   // G: NH rows, NB columns
  constexpr int RE = NB / V, SE = 256 / RE, CE = (NH + SE - 1) / SE;   // E: NB rows, NH columns
  __shared__ double yv[NB], prev[NB], zn[NH], pd[SD][NB], pg[SG][NH], pe[SE][NB];
  const int w = blockIdx.x, t = threadIdx.x;
  const int g0 = h.win_off[w], g1 = h.win_off[w + 1];
  if (g1 <= g0) return;
  const int d0 = (t % RD) * V, dq = t / RD;                   // first row / column slice: D^-1
  const int gr0 = (t % RG) * V, gq = t / RG;                  // G
  const int e0 = (t % RE) * V, eq = t / RE;                   // E
  const bool dON = t < SD * RD, gON = t < SG * RG, eON = t < SE * RE;
  // The window slot of this thread's row is loaded a super-row before the vector value it
  // addresses, and both before the factor prefetch: the vector memory counter completes in
  // order, so waiting for a slot issued after the prefetch would wait for the prefetch too.
  const int ta = t < NB ? t / NFF : 0;
  auto slot = [&](int g) { return h.win_slot[5 * g + ta]; };
  auto own = [&](int g) { return h.win_own[5 * g + ta]; };
  auto xat = [&](int f) -> double { return (t < NB && f >= 0) ? x[(size_t)f * NFF + t % NFF] : 0.0; };
  T gr[CG][V], dr[CD][V];
  // lanes without an entry read the block's first entry, which the products multiply by
  // zero: selecting zero right after the load would wait for it and stall the prefetch
  auto load_fwd = [&](int g) {
    const T* Gg = Wg + (size_t)g * NH * NB;                  // Gg[k * NH + i] = G_r[i][k]
    const T* Dg = Wd + (size_t)g * NB * NB;                  // Dg[k * NB + i] = D_r^-1[i][k]
#pragma unroll
    for (int kk = 0; kk < CG; ++kk) {
      const int k = gq * CG + kk;
      const bool ok = gON && g > g0 && k < NB;
      L::get(Gg + (ok ? (size_t)k * NH + gr0 : 0), gr[kk]);
    }
#pragma unroll
    for (int kk = 0; kk < CD; ++kk) {
      const int k = dq * CD + kk;
      const bool ok = dON && k < NB;
      L::get(Dg + (ok ? (size_t)k * NB + d0 : 0), dr[kk]);
    }
  };
  double xn = xat(slot(g0));
  int sn = slot(g0 + 1 < g1 ? g0 + 1 : g0);                 // slot of the next super-row
  load_fwd(g0);
  for (int g = g0; g < g1; ++g) {
    if (t < NB) yv[t] = xn;
    lds_barrier();
    T gc[CG][V], dc[CD][V];
#pragma unroll
    for (int kk = 0; kk < CG; ++kk)
#pragma unroll
      for (int v = 0; v < V; ++v) gc[kk][v] = gr[kk][v];
#pragma unroll
    for (int kk = 0; kk < CD; ++kk)
#pragma unroll
      for (int v = 0; v < V; ++v) dc[kk][v] = dr[kk][v];
    // (the slot loads are unconditional, with the index clamped, so that the loaded
    // register is the loop-carried one and no copy waits for it)
    const int s1 = sn;
    sn = slot(g + 2 < g1 ? g + 2 : g);
    if (g + 1 < g1) {
      xn = xat(s1);
      load_fwd(g + 1);
    }
    if (g > g0) {
      if (gON) {
        double a[V];
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] = 0.0;
#pragma unroll
        for (int kk = 0; kk < CG; ++kk) {
          const int k = gq * CG + kk;
          const double pk = k < NB ? prev[k] : 0.0;
#pragma unroll
          for (int v = 0; v < V; ++v) a[v] += (double)gc[kk][v] * pk;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) pg[gq][gr0 + v] = a[v];
      }
      lds_barrier();
      if (t < NH) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < SG; ++q) a += pg[q][t];
        yv[t] -= a;
      }
      lds_barrier();
    }
    if (dON) {
      double a[V];
#pragma unroll
      for (int v = 0; v < V; ++v) a[v] = 0.0;
#pragma unroll
      for (int kk = 0; kk < CD; ++kk) {
        const int k = dq * CD + kk;
        const double yk = k < NB ? yv[k] : 0.0;
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] += (double)dc[kk][v] * yk;
      }
#pragma unroll
      for (int v = 0; v < V; ++v) pd[dq][d0 + v] = a[v];
    }
    if (t < NB) prev[t] = yv[t];
    lds_barrier();
    if (t < NB) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < SD; ++q) a += pd[q][t];
      Wy[(size_t)g * D::NSV + NB + t] = a;                   // w_r, read back by this thread
    }
  }
  // backward sweep
  T er[CE][V];
  auto load_bwd = [&](int g) {
    const T* Eg = Wc + (size_t)g * NB * NH;                  // Eg[k * NB + i] = E_r[i][k]
#pragma unroll
    for (int kk = 0; kk < CE; ++kk) {
      const int k = eq * CE + kk;
      const bool ok = eON && k < NH;
      L::get(Eg + (ok ? (size_t)k * NB + e0 : 0), er[kk]);
    }
  };
  // slot and ownership of the super-row, loaded a step ahead (before the E prefetch)
  int bs = slot(g1 - 1), bo = own(g1 - 1);
  if (g1 - 2 >= g0) load_bwd(g1 - 2);
  for (int g = g1 - 1; g >= g0; --g) {
    const int fs = bs, fo = bo;
    double v = t < NB ? Wy[(size_t)g * D::NSV + NB + t] : 0.0;
    bs = slot(g - 1 >= g0 ? g - 1 : g);
    bo = own(g - 1 >= g0 ? g - 1 : g);
    if (g < g1 - 1) {
      T ec[CE][V];
#pragma unroll
      for (int kk = 0; kk < CE; ++kk)
#pragma unroll
        for (int u = 0; u < V; ++u) ec[kk][u] = er[kk][u];
      if (g - 1 >= g0) load_bwd(g - 1);
      if (eON) {
        double a[V];
#pragma unroll
        for (int u = 0; u < V; ++u) a[u] = 0.0;
#pragma unroll
        for (int kk = 0; kk < CE; ++kk) {
          const int k = eq * CE + kk;
          const double zk = k < NH ? zn[k] : 0.0;
#pragma unroll
          for (int u = 0; u < V; ++u) a[u] += (double)ec[kk][u] * zk;
        }
#pragma unroll
        for (int u = 0; u < V; ++u) pe[eq][e0 + u] = a[u];
      }
      lds_barrier();
      if (t < NB) {
#pragma unroll
        for (int q = 0; q < SE; ++q) v -= pe[q][t];
      }
    }
    lds_barrier();                                           // zn and pe free again
    if (t < NB) {
      if (t < NH) zn[t] = v;
      if (fs >= 0 && fo) z[(size_t)fs * NFF + t % NFF] = v;
    }
    lds_barrier();
  }
}

// y = S x: one 64-lane workgroup per facet over the NFF rows of S_T on both sides.  The wave
// covers four rows at a time with 16 lanes per row on consecutive columns (four 64-byte
// segments per load), so a row's sum is reduced over 16 lanes (4 shuffle steps) instead
// of the whole wave.
template <int K, class T>
__global__ void __launch_bounds__(64) facet_apply_kernel(DeviceHDG h, const T* __restrict__ blk, size_t bs,
                                                         const double* __restrict__ x, double* __restrict__ y) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  constexpr int RG = NFF / 4, CB = NF / 16;                 // row quads, 16-column blocks
  static_assert(NFF % 4 == 0 && NF % 16 == 0, "facet block shape");
  __shared__ double xs[2][NF];
  const int hf = blockIdx.x, tid = threadIdx.x;
  const int rq = tid >> 4, cl = tid & 15;
  int pe[2], fc[2];
  for (int s = 0; s < 2; ++s) {
    pe[s] = h.hf_side[2 * hf + s];
    fc[s] = h.hf_face[2 * hf + s];
  }
  for (int s = 0; s < 2; ++s)
    for (int i = tid; i < NF; i += 64)
      xs[s][i] = (pe[s] >= 0) ? x[(size_t)h.efacet[4 * pe[s] + i / NFF] * NFF + i % NFF] : 0.0;
  __syncthreads();
  double acc[RG];
#pragma unroll
  for (int r = 0; r < RG; ++r) acc[r] = 0.0;
  for (int s = 0; s < 2; ++s) {
    if (pe[s] < 0) continue;
    const T* Sb = blk + (size_t)pe[s] * bs + (size_t)(NU + fc[s] * NFF) * NC + NU;   // NFF rows of S_T
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int c = 16 * cb + cl;
      const double xc = xs[s][c];
#pragma unroll
      for (int r = 0; r < RG; ++r) acc[r] += (double)Sb[(size_t)(4 * r + rq) * NC + c] * xc;
    }
  }
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    double v = acc[r];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (cl == 0) y[(size_t)hf * NFF + 4 * r + rq] = v;
  }
}

// ---------------------------------------------------------------------------
// device-resident GMRES pieces
// ---------------------------------------------------------------------------
constexpr int GM_NB = 256;        // blocks of the reduction kernels
constexpr int GM_MAXM = 64;       // maximum restart length

struct GmState {                  // device layout of the small GMRES arrays (doubles)
  static constexpr int H = 0;                                   // (MAXM+1) x MAXM column-major: H[j*(MAXM+1)+i]
  static constexpr int CS = H + (GM_MAXM + 1) * GM_MAXM;
  static constexpr int SN = CS + GM_MAXM;
  static constexpr int G = SN + GM_MAXM;                        // MAXM+1
  static constexpr int RES = G + GM_MAXM + 1;                   // residual estimates |g_{j+1}|
  static constexpr int HC = RES + GM_MAXM;                      // current column dots (MAXM+1)
  static constexpr int INVB = HC + GM_MAXM + 1;                 // 1 / beta of the newest vector
  static constexpr int PART = INVB + 2;                         // GM_NB x (MAXM+1) partial sums
  static constexpr int NPART = PART + GM_NB * (GM_MAXM + 1);    // GM_NB partial norms
  static constexpr int PART2 = NPART + GM_NB;                   // GM_NB x (MAXM+1) partial dots, second pass
  static constexpr int SIZE = PART2 + GM_NB * (GM_MAXM + 1);
};

// sum over the 64 lanes of a wave (lane 0 holds the result)
__device__ inline double gm_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// sum of the GM_NB partial norms, by one wave (every lane returns it)
__device__ inline double gm_norm_total(const double* __restrict__ st, int nblocks) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += st[GmState::NPART + b];
  s = gm_wave_sum(s);
  return __shfl(s, 0, 64);
}

// block-wide sum of one value per thread (256 threads); thread 0 gets the result
__device__ inline double gm_block_sum(double v, double* red4) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = gm_wave_sum(v);
  if (lane == 0) red4[wv] = v;
  __syncthreads();
  return red4[0] + red4[1] + red4[2] + red4[3];
}

// partial dots of w with V_0..V_{k-1}: part[b][c] (block b covers one contiguous chunk)
__global__ void __launch_bounds__(256) gm_dots_kernel(int n, int k, const double* __restrict__ V, size_t ldv,
                                                      const double* __restrict__ w, double* __restrict__ st) {
  __shared__ double red[4][8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int chunk = (n + GM_NB - 1) / GM_NB;
  const int r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  double* part = st + GmState::PART + (size_t)blockIdx.x * (GM_MAXM + 1);
  for (int c0 = 0; c0 < k; c0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = r0 + tid; r < r1; r += 256) {
      const double wr = w[r];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c0 + c < k) acc[c] += V[(size_t)(c0 + c) * ldv + r] * wr;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double t = gm_wave_sum(acc[c]);
      if (lane == 0) red[wv][c] = t;
    }
    __syncthreads();
    if (tid < 8 && c0 + tid < k) part[c0 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
}

// Classical Gram-Schmidt pass on w: h = sum of the block partials of V^T w (added into
// column j of H), w -= V h.  The first pass (pass 0, partials in PART) also forms the
// partials of the second pass's dots V^T w over the rows it has just updated (into
// PART2, so that no block overwrites partials another block is still reading); the
// second pass (pass 1, partials in PART2) forms the partials of |w|^2.
__global__ void __launch_bounds__(256) gm_orth_kernel(int n, int k, int j, const double* __restrict__ V, size_t ldv,
                                                      double* __restrict__ w, double* __restrict__ st, int pass) {
  __shared__ double hc[GM_MAXM + 1];
  __shared__ double red[4][8];
  __shared__ double red4[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int src = pass == 0 ? GmState::PART : GmState::PART2;
  for (int c = wv; c < k; c += 4) {
    double a = 0.0;
    for (int b = lane; b < GM_NB; b += 64) a += st[src + (size_t)b * (GM_MAXM + 1) + c];
    a = gm_wave_sum(a);
    if (lane == 0) hc[c] = a;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid < k) st[GmState::H + (size_t)j * (GM_MAXM + 1) + tid] += hc[tid];
  const int stride = gridDim.x * blockDim.x;
  double nrm = 0.0;
  for (int r = blockIdx.x * blockDim.x + tid; r < n; r += stride) {
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += V[(size_t)c * ldv + r] * hc[c];
    const double v = w[r] - acc;
    w[r] = v;
    nrm += v * v;
  }
  if (pass == 1) {
    const double t = gm_block_sum(nrm, red4);
    if (tid == 0) st[GmState::NPART + blockIdx.x] = t;
    return;
  }
  // second-pass dots over this thread's rows (each thread rereads only what it wrote)
  double* part = st + GmState::PART2 + (size_t)blockIdx.x * (GM_MAXM + 1);
  for (int c0 = 0; c0 < k; c0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = blockIdx.x * blockDim.x + tid; r < n; r += stride) {
      const double wr = w[r];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c0 + c < k) acc[c] += V[(size_t)(c0 + c) * ldv + r] * wr;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double t = gm_wave_sum(acc[c]);
      if (lane == 0) red[wv][c] = t;
    }
    __syncthreads();
    if (tid < 8 && c0 + tid < k) part[c0 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
}

// |w|^2 partials only (for the initial residual)
__global__ void __launch_bounds__(256) gm_norm_kernel(int n, const double* __restrict__ w, double* __restrict__ st) {
  __shared__ double red4[4];
  const int tid = threadIdx.x;
  double nrm = 0.0;
  for (int r = blockIdx.x * blockDim.x + tid; r < n; r += gridDim.x * blockDim.x) nrm += w[r] * w[r];
  const double t = gm_block_sum(nrm, red4);
  if (tid == 0) st[GmState::NPART + blockIdx.x] = t;
}

// start a cycle: beta = |r|, g = (beta, 0, ...), H = 0, invb = 1/beta
// hbeta: host-visible copy of beta (coherent pinned memory), read by the host after the
// block that follows
__global__ void gm_start_kernel(double* __restrict__ st, int nblocks, double* __restrict__ hbeta) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const double beta = sqrt(gm_norm_total(st, nblocks));
    if (tid == 0) {
      st[GmState::G] = beta;
      st[GmState::INVB] = beta > 0.0 ? 1.0 / beta : 0.0;
      st[GmState::INVB + 1] = beta;
      *hbeta = beta;
    }
  }
  for (int i = tid; i < (GM_MAXM + 1) * GM_MAXM; i += blockDim.x) st[GmState::H + i] = 0.0;
  for (int i = 1 + tid; i < GM_MAXM + 1; i += blockDim.x) st[GmState::G + i] = 0.0;
}

// Givens update of column j and v /= beta in one launch: every block sums the norm
// partials itself (beta is needed everywhere); block 0 also updates the rotations.
// hres: host-visible residual estimates (coherent pinned memory), hres[j] written with RES[j]
__global__ void __launch_bounds__(256) gm_givens_scale_kernel(int n, int j, double* __restrict__ v,
                                                              double* __restrict__ st, int nblocks,
                                                              double* __restrict__ hres) {
  __shared__ double sb[1];
  if (threadIdx.x < 64) {
    const double beta = sqrt(gm_norm_total(st, nblocks));
    if (threadIdx.x == 0) sb[0] = beta;
  }
  __syncthreads();
  const double beta = sb[0];
  const double inv = (beta > 1e-300) ? 1.0 / beta : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* Hc = st + GmState::H + (size_t)j * (GM_MAXM + 1);
    Hc[j + 1] = beta;
    for (int i = 0; i < j; ++i) {
      const double c = st[GmState::CS + i], sn = st[GmState::SN + i];
      const double t = c * Hc[i] + sn * Hc[i + 1];
      Hc[i + 1] = -sn * Hc[i] + c * Hc[i + 1];
      Hc[i] = t;
    }
    const double a = Hc[j], b = Hc[j + 1];
    const double rr = sqrt(a * a + b * b);
    const double c = rr > 0.0 ? a / rr : 1.0, sn = rr > 0.0 ? b / rr : 0.0;
    st[GmState::CS + j] = c;
    st[GmState::SN + j] = sn;
    Hc[j] = rr;
    Hc[j + 1] = 0.0;
    const double gj = st[GmState::G + j];
    st[GmState::G + j + 1] = -sn * gj;
    st[GmState::G + j] = c * gj;
    st[GmState::RES + j] = fabs(sn * gj);
    hres[j] = fabs(sn * gj);
    st[GmState::INVB] = inv;
  }
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] *= inv;
}

__global__ void gm_scale_copy_kernel(int n, const double* __restrict__ x, double* __restrict__ v,
                                     const double* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = x[i] * st[GmState::INVB];
}

// least squares of the Arnoldi cycle on the device: H[0:k, 0:k] y = g[0:k], H already
// rotated to upper triangular (one thread: k <= 64)
__global__ void gm_lsq_kernel(int k, const double* __restrict__ st, double* __restrict__ y) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double* H = st + GmState::H;
  const double* g = st + GmState::G;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int q = i + 1; q < k; ++q) s -= H[(size_t)q * (GM_MAXM + 1) + i] * y[q];
    const double d = H[(size_t)i * (GM_MAXM + 1) + i];
    y[i] = (d != 0.0) ? s / d : 0.0;
  }
}

// r = V y (y on the device, length k)
__global__ void gm_combine_kernel(int n, int k, const double* __restrict__ V, size_t ldv,
                                  const double* __restrict__ y, double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int c = 0; c < k; ++c) acc += V[(size_t)c * ldv + i] * y[c];
  r[i] = acc;
}

// y += a x
__global__ void axpy_kernel(int n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// r = b - r
__global__ void rsub_kernel(int n, const double* __restrict__ b, double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - r[i];
}

__global__ void zero_kernel(int n, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// back-substitution: dU = -K^-1 f - K^-1 C dUhat; U += dU on implicit elements; max |dU|, max |U| per block.
// 16 lanes per row of X on consecutive columns, 16 rows at a time over the 256 threads, each
// row's sum reduced over its 16 lanes.
template <int K, class T>
__global__ void __launch_bounds__(256) hdg_backsub_kernel(DeviceHDG h, const T* __restrict__ X,
                                                          const double* __restrict__ dUh, double* __restrict__ U,
                                                          double* __restrict__ part) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP;
  constexpr int RP = (NU + 15) / 16, CB = NF / 16;          // row passes, 16-column blocks
  static_assert(NF % 16 == 0, "facet columns");
  __shared__ double xs[NF];
  __shared__ double rd[2][256];
  const int p = blockIdx.x;
  const int e = h.im_list[p];
  const int tid = threadIdx.x, rq = tid >> 4, cl = tid & 15;
  for (int i = tid; i < NF; i += blockDim.x) xs[i] = dUh[(size_t)h.efacet[4 * p + i / NFF] * NFF + i % NFF];
  __syncthreads();
  double xv[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) xv[cb] = xs[16 * cb + cl];
  double mdu = 0.0, mu = 0.0;
#pragma unroll
  for (int rp = 0; rp < RP; ++rp) {
    const int i = 16 * rp + rq;
    const bool ok = i < NU;
    const T* Xr = X + ((size_t)p * NU + (ok ? i : 0)) * (NF + 1);   // [K^-1 C | K^-1 f]
    double acc = cl == 0 ? (double)Xr[NF] : 0.0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc += (double)Xr[16 * cb + cl] * xv[cb];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (ok && cl == 0) {
      const double du = -acc;
      const double un = U[(size_t)e * NU + i] + du;
      U[(size_t)e * NU + i] = un;
      // non-finite values count as infinite (fmax would drop a NaN): the host reports them
      mdu = fmax(mdu, isfinite(du) ? fabs(du) : INFINITY);
      mu = fmax(mu, isfinite(un) ? fabs(un) : INFINITY);
    }
  }
  rd[0][tid] = mdu;
  rd[1][tid] = mu;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) { rd[0][tid] = fmax(rd[0][tid], rd[0][tid + s]); rd[1][tid] = fmax(rd[1][tid], rd[1][tid + s]); }
    __syncthreads();
  }
  if (tid == 0) { part[2 * p] = rd[0][0]; part[2 * p + 1] = rd[1][0]; }
}

// Newton increment norms: the maxima of the per-block partials of the back-substitution
// (n_im pairs: max |dU|, max |U|) and of the facet update (nf pairs: max |dUhat|, max |Uhat|),
// written to host-visible memory, the last one after a system-scope fence (the host waits
// for it).  The partials are >= 0 or infinite (non-finite values are counted as infinite).
__global__ void __launch_bounds__(256) newton_norms_kernel(int n_im, int nf, const double* __restrict__ part,
                                                           double* __restrict__ hout) {
  __shared__ double r[4][256];
  const int t = threadIdx.x;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = t; i < n_im; i += 256) {
    a[0] = fmax(a[0], part[2 * i]);
    a[1] = fmax(a[1], part[2 * i + 1]);
  }
  for (int i = t; i < nf; i += 256) {
    a[2] = fmax(a[2], part[2 * (n_im + i)]);
    a[3] = fmax(a[3], part[2 * (n_im + i) + 1]);
  }
  for (int k = 0; k < 4; ++k) r[k][t] = a[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st)
      for (int k = 0; k < 4; ++k) r[k][t] = fmax(r[k][t], r[k][t + st]);
    __syncthreads();
  }
  if (t == 0) {
    hout[0] = r[0][0];
    hout[1] = r[1][0];
    hout[2] = r[2][0];
    __threadfence_system();
    hout[3] = r[3][0];
  }
}

// Uhat += dUhat; per-block max |dUhat|, max |Uhat|
__global__ void __launch_bounds__(256) facet_update_kernel(int n, const double* __restrict__ d, double* __restrict__ x,
                                                           double* __restrict__ part) {
  __shared__ double rd[2][256];
  const int tid = threadIdx.x;
  double md = 0.0, mx = 0.0;
  for (int i = blockIdx.x * blockDim.x + tid; i < n; i += gridDim.x * blockDim.x) {
    const double xn = x[i] + d[i];
    x[i] = xn;
    md = fmax(md, isfinite(d[i]) ? fabs(d[i]) : INFINITY);
    mx = fmax(mx, isfinite(xn) ? fabs(xn) : INFINITY);
  }
  rd[0][tid] = md;
  rd[1][tid] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) { rd[0][tid] = fmax(rd[0][tid], rd[0][tid + s]); rd[1][tid] = fmax(rd[1][tid], rd[1][tid + s]); }
    __syncthreads();
  }
  if (tid == 0) { part[2 * blockIdx.x] = rd[0][0]; part[2 * blockIdx.x + 1] = rd[1][0]; }
}

// ---------------------------------------------------------------------------
// Transposed stage system (reverse mode of the implicit stage, Sec. 4.3).  With
// J = [[K C],[D E]] per element (HDG-MX: mixed block eliminated) and facet rows
// assembled over the elements, J^T [lam; lamhat] = [a; ahat] is condensed as
//   w = K^-T a,   S^T lamhat = ahat - sum_T C_T^T w_T,   lam = K^-T (a - D^T lamhat)
// (S^T = E^T - C^T K^-T D^T), reusing K^-1 and the condensed blocks of the forward
// path.  Element vectors use the full-state layout [e][v][n] (rows of implicit
// elements), facet vectors the Uhat layout.
// ---------------------------------------------------------------------------

// out_e = K^-T in_e on implicit elements
template <int K, class T>
__global__ void __launch_bounds__(128) kinvT_kernel(DeviceHDG h, const T* __restrict__ Kinv,
                                                    const double* __restrict__ in, double* __restrict__ out) {
  constexpr int NU = 4 * (K + 1) * (K + 1);
  __shared__ double a[NU];
  const int p = blockIdx.x, tid = threadIdx.x;
  const size_t e = h.im_list[p];
  for (int i = tid; i < NU; i += blockDim.x) a[i] = in[e * NU + i];
  __syncthreads();
  const T* Kp = Kinv + (size_t)p * NU * NU;
  for (int n = tid; n < NU; n += blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < NU; ++m) acc += (double)Kp[(size_t)m * NU + n] * a[m];
    out[e * NU + n] = acc;
  }
}

// out_F += coef sum_T (C_T^T v_T)|_F, v on implicit elements (full-state layout)
template <int K, class T>
__global__ void facet_CT_kernel(DeviceHDG h, size_t bs, const T* __restrict__ blk, const double* __restrict__ v,
                                double coef, double* __restrict__ out) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * NFF) return;
  const int hf = t / NFF, j = t % NFF;
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * hf + s];
    if (pe < 0) continue;
    const int lf = h.hf_face[2 * hf + s];
    const T* B = blk + (size_t)pe * bs + NU + lf * NFF + j;
    const double* vv = v + (size_t)h.im_list[pe] * NU;
    for (int m = 0; m < NU; ++m) acc += (double)B[(size_t)m * NC] * vv[m];
  }
  out[t] += coef * acc;
}

// y = S^T x on the facets
template <int K, class T>
__global__ void facet_applyT_kernel(DeviceHDG h, size_t bs, const T* __restrict__ blk, const double* __restrict__ x,
                                    double* __restrict__ y) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * NFF) return;
  const int hf = t / NFF, j = t % NFF;
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * hf + s];
    if (pe < 0) continue;
    const int lf = h.hf_face[2 * hf + s];
    const T* B = blk + (size_t)pe * bs + (size_t)NU * NC + NU + lf * NFF + j;      // column (lf, j) of S_T
    for (int lg = 0; lg < 4; ++lg) {
      const double* xg = x + (size_t)h.efacet[4 * pe + lg] * NFF;
      for (int i = 0; i < NFF; ++i) acc += (double)B[(size_t)(lg * NFF + i) * NC] * xg[i];
    }
  }
  y[t] = acc;
}

// lam_e = K^-T (a_e - D_T^T lamhat_T) on implicit elements
template <int K, class T>
__global__ void __launch_bounds__(128) backsubT_kernel(DeviceHDG h, size_t bs, const T* __restrict__ blk,
                                                       const T* __restrict__ Kinv, const double* __restrict__ a,
                                                       const double* __restrict__ lh, double* __restrict__ lam) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  __shared__ double xs[NF], tv[NU];
  const int p = blockIdx.x, tid = threadIdx.x;
  const size_t e = h.im_list[p];
  for (int i = tid; i < NF; i += blockDim.x) xs[i] = lh[(size_t)h.efacet[4 * p + i / NFF] * NFF + i % NFF];
  __syncthreads();
  const T* B = blk + (size_t)p * bs;
  for (int m = tid; m < NU; m += blockDim.x) {
    double acc = a[e * NU + m];
    for (int i = 0; i < NF; ++i) acc -= (double)B[(size_t)(NU + i) * NC + m] * xs[i];
    tv[m] = acc;
  }
  __syncthreads();
  const T* Kp = Kinv + (size_t)p * NU * NU;
  for (int n = tid; n < NU; n += blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < NU; ++m) acc += (double)Kp[(size_t)m * NU + n] * tv[m];
    lam[e * NU + n] = acc;
  }
}

// Block-Jacobi preconditioner of S^T: P_F = ((sum_T S_T[F, F])^T)^-1 per facet (FP64)
template <int K, class T>
__global__ void __launch_bounds__(64) bjT_factor_kernel(DeviceHDG h, size_t bs, const T* __restrict__ blk,
                                                        double* __restrict__ P) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP, NC = NU + NF + 1;
  using G = GJ<NFF, double>;
  __shared__ GJShared<NFF, double> sh;
  const int hf = blockIdx.x, tid = threadIdx.x;
  const bool own = G::owns(tid);
  const int r0 = G::row0(tid), c0 = G::col0(tid);
  double A[G::RT][G::CT];
#pragma unroll
  for (int i = 0; i < G::RT; ++i)
#pragma unroll
    for (int j = 0; j < G::CT; ++j) {
      double acc = 0.0;
      if (own)
        for (int s = 0; s < 2; ++s) {
          const int pe = h.hf_side[2 * hf + s];
          if (pe < 0) continue;
          const int lf = h.hf_face[2 * hf + s];
          // (S_FF)^T [r0+i][c0+j] = S_FF[c0+j][r0+i]
          acc += (double)blk[(size_t)pe * bs + (size_t)(NU + lf * NFF + c0 + j) * NC + NU + lf * NFF + r0 + i];
        }
      A[i][j] = acc;
    }
  G::invert(A, sh, tid);
  if (!own) return;
  double* Pf = P + (size_t)hf * NFF * NFF;
#pragma unroll
  for (int i = 0; i < G::RT; ++i)
#pragma unroll
    for (int j = 0; j < G::CT; ++j) Pf[(size_t)sh.pos[r0 + i] * NFF + sh.rp[c0 + j]] = A[i][j];
}

template <int K>
__global__ void bjT_apply_kernel(int n_hf, const double* __restrict__ P, const double* __restrict__ x,
                                 double* __restrict__ y) {
  constexpr int NFF = 4 * (K + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_hf * NFF) return;
  const int hf = t / NFF, i = t % NFF;
  const double* Pr = P + ((size_t)hf * NFF + i) * NFF;
  const double* xf = x + (size_t)hf * NFF;
  double acc = 0.0;
  for (int j = 0; j < NFF; ++j) acc += Pr[j] * xf[j];
  y[t] = acc;
}

// out_e += (K_T - M_T)^T v_e / (dt_a dts_e): adjoint of R^HDG's element rows through U
template <int K, class T>
__global__ void __launch_bounds__(128) elem_KT_kernel(DeviceMesh m, DeviceHDG h, size_t bs, const T* __restrict__ blk,
                                                      double dt_a, const double* __restrict__ v,
                                                      double* __restrict__ out) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NC = NU + NF + 1;
  __shared__ double a[NU];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int e = h.im_list[p];
  for (int i = tid; i < NU; i += blockDim.x) a[i] = v[(size_t)e * NU + i];
  __syncthreads();
  const T* B = blk + (size_t)p * bs;
  const BasisTable& tb = *m.tab;
  const double jac = 0.25 * m.hx[e] * m.hy[e];
  const double sc = 1.0 / (dt_a * elem_dt(m, e));
  for (int n = tid; n < NU; n += blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < NU; ++r) acc += (double)B[(size_t)r * NC + n] * a[r];
    const int nn = n % NN;
    acc -= tb.NW[nn % NP] * tb.NW[nn / NP] * jac * a[n];
    out[(size_t)e * NU + n] += sc * acc;
  }
}

// Adjoint of the interface Dirichlet rows int_F (Uhat - u^ex) . muhat: the explicit
// element on the other side of each interface facet receives the transposed trace
//   ybar_e[v][n] += sum_q w_q phi_n(x_q) sum_m L_m(x_q) lamhat[F][v][m]
template <int K>
__global__ void interfaceT_kernel(DeviceMesh m, const int* __restrict__ ex_ifacet, const double* __restrict__ lh,
                                  double* __restrict__ ybar) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NFF = 4 * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * NN) return;
  const int e = t / NN, n = t % NN, a = n % NP, b = n / NP;
  if (m.imp[e]) return;
  const BasisTable& tb = *m.tab;
  double acc[4] = {0, 0, 0, 0};
  bool any = false;
  for (int f = 0; f < 4; ++f) {
    const int F = ex_ifacet[4 * e + f];
    if (F < 0) continue;
    any = true;
    const int s = f & 1;
    const double wl = (f < 2) ? 0.5 * m.hy[e] : 0.5 * m.hx[e];
    const double* lf = lh + (size_t)F * NFF;
    for (int q = 0; q < NQ; ++q) {
      const double ph = (f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b];
      const double w = tb.W[q] * wl * ph;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double lq = 0.0;
        for (int mm = 0; mm < NP; ++mm) lq += tb.L[q][mm] * lf[v * NP + mm];
        acc[v] += w * lq;
      }
    }
  }
  if (!any) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) ybar[(size_t)e * 4 * NN + v * NN + n] += acc[v];
}

// out_e = in_e / (dt_a dts_e) on implicit elements
template <int K>
__global__ void rows_scale_kernel(DeviceMesh m, DeviceHDG h, double dt_a, const double* __restrict__ in,
                                  double* __restrict__ out) {
  constexpr int NU = 4 * (K + 1) * (K + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_im * NU) return;
  const int e = h.im_list[t / NU];
  const size_t idx = (size_t)e * NU + t % NU;
  out[idx] = in[idx] / (dt_a * elem_dt(m, e));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#define HDG_DISPATCH(KV, ...)                                   \
  switch (KV) {                                                 \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;       \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;       \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;       \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;       \
    default: return hipErrorInvalidValue;                       \
  }

static bool use_mx(const imex_ctx* c) { return c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous; }

// HDG_DISPATCH for functions returning imex_status
#define HDG_DISPATCH_ST(KV, ...)                                \
  switch (KV) {                                                 \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;       \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;       \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;       \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;       \
    default: return IMEX_EINVAL;                                \
  }
static bool use_f32(const imex_ctx* c) { return c->opt.precision == IMEX_FP32_REFINE; }
static size_t la_bytes(const imex_ctx* c) { return use_f32(c) ? sizeof(float) : sizeof(double); }

// element type of the implicit linear algebra: LT = double (IMEX_FP64) or float (IMEX_FP32_REFINE)
#define LA_DISPATCH(CTX, ...)                                       \
  if (use_f32(CTX)) { using LT = float; __VA_ARGS__; }              \
  else { using LT = double; __VA_ARGS__; }

template <class T> static T* la(void* p) { return static_cast<T*>(p); }

static size_t blk_stride(const imex_ctx* c) {      // augmented local system (NU+NF) x (NU+NF+1)
  const size_t NU = 4 * c->NN, NF = 16 * c->NP;
  return (NU + NF) * (NU + NF + 1);
}
static size_t scr_stride(const imex_ctx* c) {
  if (!use_mx(c)) return 0;
  const size_t NU = 4 * c->NN, NF = 16 * c->NP, NQM = 5 * c->NN;
  return 2 * (NU + NF) * NQM;
}
static bool use_points(const imex_ctx* c) { (void)c; return true; }
static size_t rec_stride(const imex_ctx* c) {
  if (!use_points(c)) return 0;
  const size_t NQ = (3 * c->K + 2) / 2, NQV = NQ * NQ;
  if (use_mx(c)) return NQV * 8 * 9 + 4 * NQ * 8 * 13 + NQV * 12 + 4 * NQ * 12;
  return NQV * 8 * 12 + 4 * NQ * 16 * 16;
}

// GMRES vectors: V (m+1), z, r, b, dx, work
static size_t gm_vectors(const imex_ctx* c) { return (size_t)c->opt.gmres_restart + 7; }

size_t hdg_workspace_bytes(const imex_ctx* c) {
  const size_t n_im = c->n_im, NU = 4 * c->NN, NF = 16 * c->NP, NFF = 4 * c->NP, n = (size_t)c->n_hf * NFF;
  const size_t NB = 5 * NFF, NH = 2 * NFF, nsr = (size_t)std::max(c->n_superrows, 1);
  const size_t lb = la_bytes(c);
  return lb * (n_im * (blk_stride(c) + scr_stride(c) + NU * NU + NU * (NF + 1)) + nsr * (NB * NB + 2 * NH * NB)) +
         8 * (n_im * (rec_stride(c) + NF) + nsr * (2 * NB + NH) + n * (gm_vectors(c) + 1) + GmState::SIZE +
              2 * (n_im + 1024));
}

imex_status hdg_alloc(imex_ctx* c) {
  if (c->n_im == 0) return IMEX_OK;
  Workspace& w = c->ws;
  const size_t n_im = c->n_im, NU = 4 * c->NN, NF = 16 * c->NP, NFF = 4 * c->NP;
  const size_t n = (size_t)c->n_hf * NFF;
  const size_t lb = la_bytes(c);
  hipError_t e = hipMalloc(&w.blk, lb * n_im * blk_stride(c));
  if (e == hipSuccess && scr_stride(c)) e = hipMalloc(&w.scr, lb * n_im * scr_stride(c));
  if (e == hipSuccess && rec_stride(c)) e = hipMalloc(&w.rec, 8 * n_im * rec_stride(c));
  if (e == hipSuccess) e = hipMalloc(&w.hres, 8 * n_im * NF);
  if (e == hipSuccess) e = hipMalloc(&w.Kinv, lb * n_im * NU * NU);
  if (e == hipSuccess) e = hipMalloc(&w.X, lb * n_im * NU * (NF + 1));
  const size_t nsr = (size_t)std::max(c->n_superrows, 1), NB = 5 * NFF, NH = 2 * NFF;
  if (e == hipSuccess) e = hipMalloc(&w.Wd, lb * nsr * NB * NB);
  if (e == hipSuccess) e = hipMalloc(&w.Wg, lb * nsr * NH * NB);
  if (e == hipSuccess) e = hipMalloc(&w.Wc, lb * nsr * NB * NH);
  if (e == hipSuccess) e = hipMalloc(&w.Wy, 8 * nsr * (2 * NB + NH));
  if (e == hipSuccess) e = hipMalloc(&w.gm, 8 * n * gm_vectors(c));
  if (e == hipSuccess) e = hipMalloc(&w.Hp, 8 * n);
  if (e == hipSuccess) e = hipMalloc(&w.gH, 8 * (size_t)GmState::SIZE);
  if (e == hipSuccess) e = hipMalloc(&w.red, 8 * 2 * (n_im + 1024));
  if (e == hipSuccess) e = hipHostMalloc(&w.hred, 8 * ((size_t)GmState::SIZE + 2 * (n_im + 1024)), 0);
  if (e == hipSuccess && !w.hgm) {
    e = hipHostMalloc(&w.hgm, 8 * (size_t)(GM_MAXM + 6), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&w.hgm_dev), w.hgm, 0);
  }
  if (e != hipSuccess) {
    c->err = std::string("implicit workspace: ") + hipGetErrorString(e);
    return IMEX_ENOMEM;
  }
  e = ct_upload(c->K, c->tab);
  if (e != hipSuccess) {
    c->err = std::string("contraction tables: ") + hipGetErrorString(e);
    return IMEX_EDEVICE;
  }
  w.bytes += hdg_workspace_bytes(c);
  c->prec_valid = false;
  return IMEX_OK;
}

template <int KK, bool MX, bool JAC> static int asm_blocks(int n_im) {
  constexpr int EPB = asm_epb<KK, MX, JAC>();
  return (n_im + EPB - 1) / EPB;
}
template <int KK, bool MX, bool JAC> static size_t asm_shm() {
  return sizeof(double) * asm_slot_doubles<KK, MX, true>() * asm_epb<KK, MX, JAC>();
}

template <int KK, class LT>
static hipError_t launch_assemble_t(imex_ctx* c, double dt_a, const double* U, const double* Uhat, const double* rhs,
                                    int jacobian, double* Rh) {
  AsmParams prm{dt_a, c->opt.alpha_hdg, c->opt.hdg_flux == IMEX_HDG_FLUX_LF, jacobian};
  Workspace& w = c->ws;
  LT* blk = la<LT>(w.blk);
  LT* scr = la<LT>(w.scr);
  const int ta = jacobian ? c->timer_begin(TM_ASSEMBLE) : -1;
  if (use_mx(c)) {
    // point values, residual rows and point-wise Jacobians; then the block contraction
    const int tpo = jacobian ? c->timer_begin(TM_POINTS) : -1;
    if (jacobian) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, true, true, LT, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asm_shm<KK, true, true>());
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, true, true, LT, true>), dim3((asm_blocks<KK, true, true>(c->n_im))), dim3(256), (asm_shm<KK, true, true>()),
                         c->stream, c->dmesh(), c->dhdg(), c->gas, prm, U, Uhat, rhs, blk, scr, w.Q, Rh, w.rec,
                         w.hres);
    } else {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, true, true, LT, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asm_shm<KK, true, false>());
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, true, true, LT, false>), dim3((asm_blocks<KK, true, false>(c->n_im))), dim3(256), (asm_shm<KK, true, false>()),
                         c->stream, c->dmesh(), c->dhdg(), c->gas, prm, U, Uhat, rhs, blk, scr, w.Q, Rh, w.rec,
                         w.hres);
    }
    c->timer_end(tpo);
    if (jacobian) {
      const int nblk = 40 * ((c->n_im + 7) / 8);
      const int tc = c->timer_begin(TM_CONTRACT);
      hipLaunchKernelGGL((hdg_contract_kernel<KK, LT, true>), dim3(nblk), dim3(256), 0, c->stream, c->dmesh(),
                         c->dhdg(), dt_a, w.rec, blk, scr);
      c->timer_end(tc);
    }
    c->timer_end(ta);
    if (jacobian) {
      // eliminate the mixed block: [[K C],[D E]] -= [A12; A32] M_Q^-1 [A21 A23]
      constexpr int NU = 4 * (KK + 1) * (KK + 1), NF = 16 * (KK + 1), NR = NU + NF, NQM = 5 * (KK + 1) * (KK + 1);
      const int te = c->timer_begin(TM_ELIMINATE);
      const long long ss = (long long)scr_stride(c);
      const hipError_t ge = gemm_batched<LT>(c->stream, c->n_im, NR, NR, NQM, -1.0, true, scr, NQM, ss,
                                             scr + (size_t)NR * NQM, NR, ss, blk, NR + 1, (long long)blk_stride(c),
                                             c->gemm_tile[0]);
      c->timer_end(te);
      if (ge != hipSuccess) return ge;
    }
  } else if (!c->gas.viscous) {
    // inviscid HDG-IP: the same split without mixed blocks (K and C D E)
    const int tpo = jacobian ? c->timer_begin(TM_POINTS) : -1;
    if (jacobian) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, false, true, LT, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asm_shm<KK, false, true>());
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, false, true, LT, true>), dim3((asm_blocks<KK, false, true>(c->n_im))), dim3(256), (asm_shm<KK, false, true>()),
                         c->stream, c->dmesh(), c->dhdg(), c->gas, prm, U, Uhat, rhs, blk, scr, nullptr, Rh, w.rec,
                         w.hres);
    } else {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, false, true, LT, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asm_shm<KK, false, false>());
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, false, true, LT, false>), dim3((asm_blocks<KK, false, false>(c->n_im))), dim3(256), (asm_shm<KK, false, false>()),
                         c->stream, c->dmesh(), c->dhdg(), c->gas, prm, U, Uhat, rhs, blk, scr, nullptr, Rh, w.rec,
                         w.hres);
    }
    c->timer_end(tpo);
    if (jacobian) {
      const int nblk = 16 * ((c->n_im + 7) / 8);
      const int tc = c->timer_begin(TM_CONTRACT);
      hipLaunchKernelGGL((hdg_contract_kernel<KK, LT, false>), dim3(nblk), dim3(256), 0, c->stream, c->dmesh(),
                         c->dhdg(), dt_a, w.rec, blk, scr);
      c->timer_end(tc);
    }
    c->timer_end(ta);
  } else {
    // viscous HDG-IP: point records (with the gradient columns), then their contraction
    const int tpo = jacobian ? c->timer_begin(TM_POINTS) : -1;
    if (jacobian) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, false, true, LT, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asm_shm<KK, false, true>());
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, false, true, LT, true>), dim3((asm_blocks<KK, false, true>(c->n_im))), dim3(256), (asm_shm<KK, false, true>()),
                         c->stream, c->dmesh(), c->dhdg(), c->gas, prm, U, Uhat, rhs, blk, scr, nullptr, Rh, w.rec,
                         w.hres);
    } else {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, false, true, LT, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asm_shm<KK, false, false>());
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, false, true, LT, false>), dim3((asm_blocks<KK, false, false>(c->n_im))), dim3(256), (asm_shm<KK, false, false>()),
                         c->stream, c->dmesh(), c->dhdg(), c->gas, prm, U, Uhat, rhs, blk, scr, nullptr, Rh, w.rec,
                         w.hres);
    }
    c->timer_end(tpo);
    if (jacobian) {
      const int tc = c->timer_begin(TM_CONTRACT);
      hipLaunchKernelGGL((hdg_contract_ipv_kernel<KK, LT>), dim3(3 * c->n_im), dim3(256), 0, c->stream, c->dmesh(),
                         c->dhdg(), dt_a, w.rec, blk);
      c->timer_end(tc);
    }
    c->timer_end(ta);
  }
  return hipGetLastError();
}

static hipError_t launch_assemble(imex_ctx* c, double dt_a, const double* U, const double* Uhat, const double* rhs,
                                  int jacobian, double* Rh) {
  HDG_DISPATCH(c->K, { LA_DISPATCH(c, return launch_assemble_t<KK, LT>(c, dt_a, U, Uhat, rhs, jacobian, Rh)); });
  return hipErrorInvalidValue;
}

// K^-1 of every implicit element: the register Gauss-Jordan, or in FP32 with inv_method = 1
// the blocked Gauss-Jordan on the matrix cores
template <int KK, class LT>
static void launch_invert(imex_ctx* c, const LT* blk, LT* Kinv) {
  if constexpr (std::is_same<LT, float>::value) {
    if (c->inv_method == 1) {
      const size_t shm = GjiDims<KK>::LDS;
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_invert_mfma_kernel<KK>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      hipLaunchKernelGGL((hdg_invert_mfma_kernel<KK>), dim3(c->n_im), dim3(256), shm, c->stream, blk_stride(c), blk,
                         Kinv);
      return;
    }
  }
  hipLaunchKernelGGL((hdg_invert_kernel<KK, LT>), dim3(c->n_im), dim3(256), 0, c->stream, blk_stride(c), blk, Kinv);
}

// condensation (eqs. statically_condensed_system, SchurCompliment):
//   K^-1 (Gauss-Jordan);  X = K^-1 [C f];  [E h] -= D X  (so that the augmented
//   system's facet block holds S_T = E - D K^-1 C and h - D K^-1 f)
static hipError_t launch_condense(imex_ctx* c) {
  Workspace& w = c->ws;
  HDG_DISPATCH(c->K, LA_DISPATCH(c, {
    constexpr int NU = 4 * (KK + 1) * (KK + 1), NF = 16 * (KK + 1), NC = NU + NF + 1;
    LT* blk = la<LT>(w.blk);
    LT* Kinv = la<LT>(w.Kinv);
    LT* X = la<LT>(w.X);
    const int ti = c->timer_begin(TM_INVERT);
    launch_invert<KK, LT>(c, blk, Kinv);
    c->timer_end(ti);
    const long long bs = (long long)blk_stride(c);
    hipError_t e = gemm_batched<LT>(c->stream, c->n_im, NU, NF + 1, NU, 1.0, false, Kinv, NU, (long long)NU * NU,
                                    blk + NU, NC, bs, X, NF + 1, (long long)NU * (NF + 1), c->gemm_tile[1]);
    if (e != hipSuccess) return e;
    e = gemm_batched<LT>(c->stream, c->n_im, NF, NF + 1, NU, -1.0, true, blk + (size_t)NU * NC, NC, bs, X, NF + 1,
                         (long long)NU * (NF + 1), blk + (size_t)NU * NC + NU, NC, bs, c->gemm_tile[2]);
    if (e != hipSuccess) return e;
  }));
  return hipGetLastError();
}

// Right-hand side of a simplified Newton correction.  The residual assembly has put the
// new f in the augmented column of the element rows and zeroed the facet rows' column;
// The two products of a simplified correction for one element per workgroup:
// X[:, NF] = K^-1 f (f the last column of the element rows), then the facet rows' last
// column -= D X[:, NF].  16 lanes per matrix row on consecutive columns, 16 rows at a time,
// each row's sum reduced over its 16 lanes; x and K^-1 f staged in LDS (K^-1 f rounded to
// the storage type, as it is stored in X).
template <int K, class T>
__global__ void __launch_bounds__(256) resolve_kernel(size_t bs, T* __restrict__ blk, const T* __restrict__ Kinv,
                                                      T* __restrict__ X) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NC = NU + NF + 1;
  constexpr int CB = (NU + 15) / 16;                         // 16-column blocks of a row
  __shared__ double xs[NU], ys[NU];
  const int p = blockIdx.x, tid = threadIdx.x, rq = tid >> 4, cl = tid & 15;
  T* bp = blk + (size_t)p * bs;
  for (int i = tid; i < NU; i += 256) xs[i] = (double)bp[(size_t)i * NC + NU + NF];
  __syncthreads();
  const T* Kp = Kinv + (size_t)p * NU * NU;
  for (int r0 = 0; r0 < NU; r0 += 16) {
    const int i = r0 + rq;
    double acc = 0.0;
    if (i < NU) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int c = 16 * cb + cl;
        if (c < NU) acc += (double)Kp[(size_t)i * NU + c] * xs[c];
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (cl == 0 && i < NU) {
      const T y = (T)acc;
      ys[i] = (double)y;
      X[((size_t)p * NU + i) * (NF + 1) + NF] = y;
    }
  }
  __syncthreads();
  for (int r0 = 0; r0 < NF; r0 += 16) {
    const int r = r0 + rq;
    double acc = 0.0;
    if (r < NF) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int c = 16 * cb + cl;
        if (c < NU) acc += (double)bp[(size_t)(NU + r) * NC + c] * ys[c];
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (cl == 0 && r < NF) {
      T* hp = bp + (size_t)(NU + r) * NC + NU + NF;
      *hp = (T)((double)*hp - acc);
    }
  }
}

// K^-1, X[:, :NF] = K^-1 C, D and S of the previous Jacobian are untouched:
//   X[:, NF] = K^-1 f,  [h - D K^-1 f] column = -D X[:, NF]  (h is added from hres).
static hipError_t launch_resolve(imex_ctx* c) {
  Workspace& w = c->ws;
  HDG_DISPATCH(c->K, LA_DISPATCH(c, {
    LT* blk = la<LT>(w.blk);
    LT* Kinv = la<LT>(w.Kinv);
    LT* X = la<LT>(w.X);
    hipLaunchKernelGGL((resolve_kernel<KK, LT>), dim3(c->n_im), dim3(256), 0, c->stream, blk_stride(c), blk, Kinv, X);
  }));
  return hipGetLastError();
}

// average device time (ms) of reps runs of f on the context's stream
template <class F>
static float time_ms(imex_ctx* c, int reps, F&& f) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return 1e30f;
  if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); return 1e30f; }
  f();                                              // warm-up
  hipEventRecord(a, c->stream);
  for (int r = 0; r < reps; ++r) f();
  hipEventRecord(b, c->stream);
  float ms = 1e30f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 1e30f;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms / reps;
}

// Output tile of each batched GEMM (elimination, K^-1 [C f], Schur update) by timing
// both tiles on the implicit workspaces (whose contents every assembly rewrites).
imex_status hdg_autotune_gemm(imex_ctx* c) {
  if (c->n_im == 0) return IMEX_OK;
  Workspace& w = c->ws;
  HDG_DISPATCH_ST(c->K, LA_DISPATCH(c, {
    constexpr int NU = 4 * (KK + 1) * (KK + 1), NF = 16 * (KK + 1), NR = NU + NF, NC = NU + NF + 1;
    constexpr int NQM = 5 * (KK + 1) * (KK + 1);
    LT* blk = la<LT>(w.blk);
    LT* scr = la<LT>(w.scr);
    LT* Kinv = la<LT>(w.Kinv);
    LT* X = la<LT>(w.X);
    const long long bs = (long long)blk_stride(c), ss = (long long)scr_stride(c);
    for (int g = 0; g < 3; ++g) {
      if (g == 0 && !use_mx(c)) continue;
      float best = 1e30f;
      for (int tile : {64, 32, 1064, 1032, 2001, 2002, 2003, 2004, 2005, 2006, 2007, 2008, 2009, 2010, 2011}) {
        if (tile > 1000 && sizeof(LT) != 4) continue;
        if (tile > 2000 && !(g == 0 ? gemm_whole_fits(tile, NR, NR)
                                    : gemm_whole_fits(tile, g == 1 ? NU : NF, NF + 1)))
          continue;
        const float ms = time_ms(c, 3, [&]() {
          if (g == 0)
            gemm_batched<LT>(c->stream, c->n_im, NR, NR, NQM, -1.0, true, scr, NQM, ss, scr + (size_t)NR * NQM,
                             NR, ss, blk, NR + 1, bs, tile);
          else if (g == 1)
            gemm_batched<LT>(c->stream, c->n_im, NU, NF + 1, NU, 1.0, false, Kinv, NU, (long long)NU * NU, blk + NU,
                             NC, bs, X, NF + 1, (long long)NU * (NF + 1), tile);
          else
            gemm_batched<LT>(c->stream, c->n_im, NF, NF + 1, NU, -1.0, true, blk + (size_t)NU * NC, NC, bs, X,
                             NF + 1, (long long)NU * (NF + 1), blk + (size_t)NU * NC + NU, NC, bs, tile);
        });
        if (ms < best) { best = ms; c->gemm_tile[g] = tile; }
      }
    }
    if constexpr (sizeof(LT) == 4) {
      // the element inverse: register Gauss-Jordan against the blocked one on the matrix cores
      float best = 1e30f;
      int pick = 0;
      for (int m : {0, 1}) {
        c->inv_method = m;
        const float ms = time_ms(c, 3, [&]() { launch_invert<KK, LT>(c, blk, Kinv); });
        if (ms < best) { best = ms; pick = m; }
      }
      c->inv_method = pick;
    }
  }));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("GEMM autotuning: ") + hipGetErrorString(e);
    return IMEX_EDEVICE;
  }
  c->prec_valid = false;                            // the factors read the overwritten blocks
  return IMEX_OK;
}

static hipError_t launch_facet_rhs(imex_ctx* c, double* b) {
  Workspace& w = c->ws;
  const int n = c->n_hf * 4 * c->NP;
  HDG_DISPATCH(c->K, LA_DISPATCH(c, hipLaunchKernelGGL((facet_rhs_kernel<KK, LT>), dim3((n + 127) / 128), dim3(128),
                                                        0, c->stream, c->dhdg(), blk_stride(c), la<LT>(w.blk), w.hres,
                                                        b)));
  return hipGetLastError();
}

static hipError_t launch_ras_factor(imex_ctx* c) {
  Workspace& w = c->ws;
  HDG_DISPATCH(c->K, LA_DISPATCH(c, {
    constexpr int NFF = 4 * (KK + 1), NB = 5 * NFF, NH = 2 * NFF;
    // the FP32 kernel also holds the blocked Gauss-Jordan's block and tables
    const size_t shm = sizeof(LT) * ((size_t)NB * NB + 2 * (size_t)NH * NB + (size_t)NH * NH) +
                       (std::is_same<LT, float>::value ? GjbDims<NB>::BYTES : 0);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&ras_factor_kernel<KK, LT>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL((ras_factor_kernel<KK, LT>), dim3(c->n_win), dim3(256), shm, c->stream, c->dhdg(),
                       la<LT>(w.blk), blk_stride(c), la<LT>(w.Wd), la<LT>(w.Wg), la<LT>(w.Wc));
  }));
  return hipGetLastError();
}

static hipError_t launch_precond(imex_ctx* c, const double* x, double* y) {
  Workspace& w = c->ws;
  if (c->adj_mode) {
    const int n = c->n_hf * 4 * c->NP;
    HDG_DISPATCH(c->K, hipLaunchKernelGGL(bjT_apply_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                          c->n_hf, w.adj_P, x, y));
    return hipGetLastError();
  }
  const int tp = c->timer_begin(TM_PRECOND);
  HDG_DISPATCH(c->K, LA_DISPATCH(c, {
    if constexpr (KK >= 4)
      hipLaunchKernelGGL((ras_apply16_kernel<KK, LT>), dim3(c->n_win), dim3(256), 0, c->stream, c->dhdg(),
                         la<LT>(w.Wg), la<LT>(w.Wd), la<LT>(w.Wc), x, w.Wy, y);
    else
      hipLaunchKernelGGL((ras_apply_kernel<KK, LT>), dim3(c->n_win), dim3(256), 0, c->stream, c->dhdg(),
                         la<LT>(w.Wg), la<LT>(w.Wd), la<LT>(w.Wc), x, w.Wy, y);
  }));
  c->timer_end(tp);
  return hipGetLastError();
}

static hipError_t launch_apply(imex_ctx* c, const double* x, double* y) {
  if (c->adj_mode) {
    const int n = c->n_hf * 4 * c->NP;
    HDG_DISPATCH(c->K, LA_DISPATCH(c, hipLaunchKernelGGL((facet_applyT_kernel<KK, LT>), dim3((n + 127) / 128),
                                                          dim3(128), 0, c->stream, c->dhdg(), blk_stride(c),
                                                          la<LT>(c->ws.blk), x, y)));
    return hipGetLastError();
  }
  HDG_DISPATCH(c->K, LA_DISPATCH(c, hipLaunchKernelGGL((facet_apply_kernel<KK, LT>), dim3(c->n_hf), dim3(64), 0,
                                                        c->stream, c->dhdg(), la<LT>(c->ws.blk), blk_stride(c), x,
                                                        y)));
  return hipGetLastError();
}

#define HTRY(expr)                                                               \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return IMEX_EDEVICE;                                                       \
    }                                                                            \
  } while (0)

// Right-preconditioned restarted GMRES(m) on S x = b, x from 0.  The Arnoldi
// process (classical Gram-Schmidt with one re-orthogonalisation pass, Givens
// rotations) runs entirely on the device in blocks of iterations; after each block the
// host reads the block's residual estimates and, at the end, solves the small
// least-squares problem.  Iterations past convergence inside a block are wasted and a
// host check costs far less than an iteration, so the block lengths are predicted: the
// first from the iteration count of the previous solve of the same kind (less one), the
// following ones from the residual's recent contraction rate (at most GM_CHECK).
constexpr int GM_CHECK = 8;
constexpr int GM_FIRST = 4;           // first block without a history
constexpr size_t GM_MAXGRAPHS = 512;  // captured block graphs kept per context
// Replay of the inner GMRES blocks from captured graphs (1) or direct launches (0).  With
// the host waiting on the residual estimates in coherent memory, direct launches start a
// block sooner (about 20 us after the wait against 30 - 90 us for a graph launch, and new
// block keys cost a capture); the boundary layer and the ensemble measured the same or
// slightly faster without the graphs.
#ifndef GM_BLOCK_GRAPHS
#define GM_BLOCK_GRAPHS 0
#endif
// Facet preconditioner reuse: refactorise once the GMRES iterations spent above the count
// right after the last factorisation exceed what a factorisation costs, in iterations (the
// online rule that pays at most twice the best choice in hindsight).  The cost ratio is
// measured: the device time of the last factorisation over the device time per iteration
// of an earlier facet solve (its events complete once a later solve has synchronised),
// smoothed, within [PREC_COST_MIN, PREC_COST_MAX]; 8 iterations until measured.
constexpr double PREC_COST_MIN = 2.0, PREC_COST_MAX = 200.0;

static hipError_t prec_events(imex_ctx* c) {
  for (hipEvent_t* e : {&c->pev_f[0], &c->pev_f[1], &c->pev_g[0][0], &c->pev_g[0][1], &c->pev_g[1][0],
                        &c->pev_g[1][1]})
    if (!*e) {
      const hipError_t r = hipEventCreate(e);
      if (r != hipSuccess) return r;
    }
  return hipSuccess;
}

// after a facet solve returned (it synchronised the stream after every earlier event):
// read the last factorisation's time and the other slot's solve time
static void prec_cost_update(imex_ctx* c) {
  float ms = 0.0f;
  if (c->pev_fset && hipEventElapsedTime(&ms, c->pev_f[0], c->pev_f[1]) == hipSuccess) {
    c->prec_fac_ms = ms;
    c->pev_fset = false;
  }
  const int o = c->pev_slot;                          // the slot not written by the last solve
  if (c->pev_gset[o] && c->pev_gits[o] > 0 && hipEventElapsedTime(&ms, c->pev_g[o][0], c->pev_g[o][1]) == hipSuccess) {
    const double it_ms = ms / c->pev_gits[o];
    c->prec_it_ms = c->prec_it_ms > 0.0 ? 0.5 * (c->prec_it_ms + it_ms) : it_ms;
    c->pev_gset[o] = false;
  }
  if (c->prec_fac_ms > 0.0 && c->prec_it_ms > 0.0)
    c->prec_cost_its = std::min(PREC_COST_MAX, std::max(PREC_COST_MIN, c->prec_fac_ms / c->prec_it_ms));
}
// a simplified Newton correction follows only a correction that contracted by at least this
constexpr double SIMPLIFIED_QMAX = 0.05;
// relative residual of the facet solve of a simplified correction
constexpr double SIMPLIFIED_GMRES_RTOL = 1e-4;
// With gmres_forcing = 2 (3) the facet solve of the first (first two) full correction(s) of
// a stage stops at min(this, q / 100), q the contraction of the second correction against
// the first in the previous stage.  The first correction's linear error then stays a
// hundredth of the second correction; the second's is removed by the correction that
// follows it, or is below the Newton tolerance when the stage stops there.
constexpr double FIRST_CORRECTION_RTOL = 1e-5;

// Run body() (kernel launches only) on the context's stream, or, with graphs enabled,
// replay its capture for key (captured on first use; the launches of an inner GMRES
// block depend only on the block's first column and on the workspaces).
template <class F>
static imex_status replay_block(imex_ctx* c, int key, F&& body) {
  if (!c->use_graphs || c->capturing) return body();
  auto it = c->gm_graphs.find(key);
  if (it == c->gm_graphs.end()) {
    hipStream_t orig = c->stream;
    HTRY(hipStreamSynchronize(orig));
    HTRY(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeRelaxed));
    c->stream = c->gstream;
    c->capturing = true;
    const imex_status st = body();
    c->capturing = false;
    c->stream = orig;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->gstream, &graph);
    if (st != IMEX_OK) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    HTRY(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    HTRY(ei);
    it = c->gm_graphs.emplace(key, exec).first;
  }
  HTRY(hipGraphLaunch(it->second, c->stream));
  return IMEX_OK;
}

// Wait until the device has overwritten *slot (coherent host memory, holding sentinel):
// spin for up to SPIN_US microseconds, then wait for the stream.  Everything the device
// wrote before that value (earlier kernels on the stream) is visible once it is.
constexpr double SPIN_US = 10000.0;
static hipError_t wait_host_value(imex_ctx* c, const double* slot, double sentinel) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    double v;
    __atomic_load(slot, &v, __ATOMIC_ACQUIRE);
    if (!(v == sentinel)) return hipSuccess;
    const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    if (us > SPIN_US) return hipStreamSynchronize(c->stream);
  }
}

// Iterations still needed to bring the residual estimate res[n-1] below tol at the
// geometric rate of the last (up to three) iterations; res[-1] is the cycle's |r_0|.
static int gm_predict(const std::vector<double>& res, double tol) {
  const int n = (int)res.size();
  const int q = std::min(3, n - 1);
  if (q < 1) return GM_FIRST;
  const double last = res[n - 1];
  const double rate = std::pow(last / res[n - 1 - q], 1.0 / q);
  if (!(rate > 0.0 && rate < 0.999) || !(last > 0.0)) return GM_CHECK;
  const double need = std::ceil(std::log(tol / last) / std::log(rate));
  return (int)std::min<double>(GM_CHECK, std::max(1.0, need));
}

// Right-preconditioned restarted GMRES on the condensed facet system.  *reached says
// whether the relative residual estimate fell below gmres_rtol (false when gmres_maxit
// iterations ran out first); a non-finite residual returns IMEX_ENONFINITE.
static imex_status gmres(imex_ctx* c, const double* b, double* x, int* its_out, int kind, bool* reached) {
  Workspace& w = c->ws;
  const int n = c->n_hf * 4 * c->NP;
  const int m = std::min(c->opt.gmres_restart, GM_MAXM);
  const size_t ldv = n;
  double* V = w.gm;
  double* z = V + ldv * (m + 1);
  double* r = z + ldv;
  double* yd = w.gH + GmState::HC;           // reuse: coefficient vector for V y
  double* st = w.gH;
  double* hb = w.hred;
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, c->stream, n, x);
  HTRY(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  double tol = -1.0;
  int total = 0;
  *its_out = 0;
  *reached = false;
  // block lengths never exceed GM_CHECK: the graph keys below rely on it
  const int hist = c->gm_hist[kind];
  int want = hist > 1 ? std::min(hist - 1, GM_CHECK) : GM_FIRST;
  std::vector<double> res;
  while (total < c->opt.gmres_maxit) {
    // beta = |r|, V_0 = r / beta; beta is read back with the first block's residual
    // estimates (a cycle that starts below the tolerance discards that block)
    hipLaunchKernelGGL(gm_norm_kernel, dim3(GM_NB), dim3(256), 0, c->stream, n, r, st);
    hipLaunchKernelGGL(gm_start_kernel, dim3(1), dim3(256), 0, c->stream, st, GM_NB, w.hgm_dev + GM_MAXM + 1);
    hipLaunchKernelGGL(gm_scale_copy_kernel, dim3(nb), dim3(256), 0, c->stream, n, r, V, st);
    bool small = false;
    int j = 0, jdone = -1;
    while (j < m && jdone < 0 && total < c->opt.gmres_maxit) {
      const int j1 = std::min(std::min(m, j + want), j + (c->opt.gmres_maxit - total));
      auto block = [&]() -> imex_status {
        for (int jj = j; jj < j1; ++jj) {
          double* vj = V + ldv * jj;
          double* vn = V + ldv * (jj + 1);
          HTRY(launch_precond(c, vj, z));
          HTRY(launch_apply(c, z, vn));
          // CGS2: dots, first pass (with the second pass's dots), second pass (with |w|^2)
          hipLaunchKernelGGL(gm_dots_kernel, dim3(GM_NB), dim3(256), 0, c->stream, n, jj + 1, V, ldv, vn, st);
          hipLaunchKernelGGL(gm_orth_kernel, dim3(GM_NB), dim3(256), 0, c->stream, n, jj + 1, jj, V, ldv, vn, st, 0);
          hipLaunchKernelGGL(gm_orth_kernel, dim3(GM_NB), dim3(256), 0, c->stream, n, jj + 1, jj, V, ldv, vn, st, 1);
          hipLaunchKernelGGL(gm_givens_scale_kernel, dim3(nb), dim3(256), 0, c->stream, n, jj, vn, st, GM_NB,
                             w.hgm_dev);
        }
        HTRY(hipGetLastError());
        return IMEX_OK;
      };
      // the launches of a block are fixed by its first column, its length and the mode
      const int key = ((j * (GM_CHECK + 1) + (j1 - j)) << 1) + (c->adj_mode ? 1 : 0);
      const bool replay = GM_BLOCK_GRAPHS && (c->gm_graphs.count(key) || c->gm_graphs.size() < GM_MAXGRAPHS);
      // the block's kernels write the residual estimates (and gm_start_kernel beta) into
      // coherent host memory.  The host spins until the block's last estimate replaces a
      // sentinel (estimates are |.| or NaN, never -1), which it sees a few microseconds
      // after the write instead of after the runtime's stream wait; past SPIN_US it waits
      // for the stream instead, which also reports any device error.
      w.hgm[j1 - 1] = -1.0;
      const imex_status bs = replay ? replay_block(c, key, block) : block();
      if (bs != IMEX_OK) return bs;
      HTRY(wait_host_value(c, &w.hgm[j1 - 1], -1.0));
      for (int jj = j; jj < j1; ++jj) hb[jj - j] = w.hgm[jj];
      if (j == 0) {
        const double beta = w.hgm[GM_MAXM + 1];
        if (!std::isfinite(beta)) {
          c->err = "non-finite facet residual";
          return IMEX_ENONFINITE;
        }
        if (tol < 0.0) tol = c->opt.gmres_rtol * beta;
        if (!(beta > tol)) { small = true; break; }
        res.assign(1, beta);
      }
      for (int jj = j; jj < j1; ++jj) {
        if (!std::isfinite(hb[jj - j])) {
          c->err = "non-finite GMRES residual estimate";
          return IMEX_ENONFINITE;
        }
        res.push_back(hb[jj - j]);
        if (!(hb[jj - j] > tol)) { jdone = jj; break; }
      }
      total += (jdone >= 0 ? jdone + 1 : j1) - j;
      j = (jdone >= 0) ? jdone + 1 : j1;
      want = gm_predict(res, tol);
    }
    if (small) { *reached = true; break; }
    const int k = j;
    if (k == 0) break;
    hipLaunchKernelGGL(gm_lsq_kernel, dim3(1), dim3(64), 0, c->stream, k, st, yd);
    hipLaunchKernelGGL(gm_combine_kernel, dim3(nb), dim3(256), 0, c->stream, n, k, V, ldv, yd, r);
    HTRY(launch_precond(c, r, z));
    hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(256), 0, c->stream, n, 1.0, z, x);
    HTRY(hipGetLastError());
    if (jdone >= 0) { *reached = true; break; }
    if (total >= c->opt.gmres_maxit) break;
    // true residual for the next cycle: r = b - S x
    HTRY(launch_apply(c, x, r));
    hipLaunchKernelGGL(rsub_kernel, dim3(nb), dim3(256), 0, c->stream, n, b, r);
    HTRY(hipGetLastError());
  }
  *its_out = total;
  c->gm_hist[kind] = total;
  return IMEX_OK;
}

static hipError_t launch_backsub(imex_ctx* c, const double* dx, double* U, double* part) {
  HDG_DISPATCH(c->K, LA_DISPATCH(c, hipLaunchKernelGGL((hdg_backsub_kernel<KK, LT>), dim3(c->n_im), dim3(256), 0,
                                                        c->stream, c->dhdg(), la<LT>(c->ws.X), dx, U, part)));
  return hipGetLastError();
}

imex_status hdg_stage_solve(imex_ctx* c, double dt_a, const double* rhs, double* U, double* Uhat, double* R_out,
                            imex_stats* st) {
  Workspace& w = c->ws;
  const int n = c->n_hf * 4 * c->NP;
  const int m = c->opt.gmres_restart;
  double* b = w.gm + (size_t)n * (m + 3);
  double* dx = b + n;
  double* part = w.red;
  const int fb = 256;
  int newton = 0, gm_total = 0;
  bool converged = false;
  double last = 0.0;
  // Newton (Sec. 4.3).  The Schwarz preconditioner of the facet solve is kept across
  // Newton iterations, stages and steps (GMRES always solves the current system); it is
  // refactorised when dt a_ii changes by more than 25 % or when the extra GMRES work
  // since the last refactorisation outweighs a new one.  Stopping: the increments of U
  // and Uhat are below rtol times the largest |U| and |Uhat|, either measured or
  // predicted from the observed contraction (theta / (1 - theta) |dz| with theta < 1/2).
  //
  // Simplified corrections (newton_simplified > 0) reuse the condensed factors of the last
  // Jacobian with a fresh FP64 residual; the increment test below is applied to them in
  // the same way, so a simplified correction that passes it certifies convergence.
  double du_prev = 0.0, dh_prev = 0.0;
  int nfull = 0;
  double q_last = 0.0;                      // contraction of the last correction
  double q2 = 0.0;                          // contraction of the second correction
  double dz_prev = 1.0;                     // relative size of the last correction
  const int need_full = c->opt.newton_simplified == 2 ? 1 : 2;
  int gm_capped = 0;                        // corrections whose facet solve hit gmres_maxit
  if (c->prec_valid && std::fabs(dt_a / c->prec_dt_a - 1.0) > 0.25) c->prec_valid = false;
  for (int it = 1; it <= c->opt.newton_maxit; ++it) {
    newton = it;
    const bool simplified = c->opt.newton_simplified > 0 && nfull >= need_full && q_last < SIMPLIFIED_QMAX;
    int tt;
    if (simplified) {
      HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 0, nullptr));
      tt = c->timer_begin(TM_CONDENSE);
      HTRY(launch_resolve(c));
      c->timer_end(tt);
    } else {
      HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 1, nullptr));
      tt = c->timer_begin(TM_CONDENSE);
      HTRY(launch_condense(c));
      c->timer_end(tt);
      ++nfull;
    }
    tt = c->timer_begin(TM_FACET);
    HTRY(launch_facet_rhs(c, b));
    if (!c->prec_valid) {
      HTRY(prec_events(c));
      HTRY(hipEventRecord(c->pev_f[0], c->stream));
      HTRY(launch_ras_factor(c));
      HTRY(hipEventRecord(c->pev_f[1], c->stream));
      c->pev_fset = true;
      c->prec_valid = true;
      c->prec_fresh = true;
      c->prec_dt_a = dt_a;
    }
    c->timer_end(tt);
    int its = 0;
    bool gm_reached = false;
    // forcing term: loose facet solves while the Newton corrections are large.  A
    // simplified correction needs only a few digits: it certifies convergence through its
    // size relative to the previous correction, and its own error (1e-4 of an increment
    // already near the tolerance) is far below the Newton tolerance.
    const double rtol = c->opt.gmres_rtol;
    if (c->opt.gmres_forcing == 1)
      c->opt.gmres_rtol = std::max(rtol, std::min(1e-4, it == 1 ? 1e-4 : 1e-2 * dz_prev));
    else if (c->opt.gmres_forcing >= 2 && (it == 1 || (it == 2 && c->opt.gmres_forcing == 3)) && !simplified &&
             c->newton_q2 > 0.0)
      c->opt.gmres_rtol = std::max(rtol, std::min(FIRST_CORRECTION_RTOL, 1e-2 * c->newton_q2));
    if (simplified) c->opt.gmres_rtol = std::max(c->opt.gmres_rtol, SIMPLIFIED_GMRES_RTOL);
    tt = c->timer_begin(TM_GMRES);
    const int slot = c->pev_slot;
    if (c->pev_g[slot][0]) HTRY(hipEventRecord(c->pev_g[slot][0], c->stream));
    imex_status s = gmres(c, b, dx, &its, simplified ? 0 : std::min(it, 4), &gm_reached);
    if (c->pev_g[slot][0]) {
      HTRY(hipEventRecord(c->pev_g[slot][1], c->stream));
      c->pev_gset[slot] = true;
      c->pev_gits[slot] = its;
      c->pev_slot = 1 - slot;
    }
    c->timer_end(tt);
    c->opt.gmres_rtol = rtol;
    if (s != IMEX_OK) return s;
    gm_total += its;
    prec_cost_update(c);
    // refactorise once the GMRES iterations spent above the post-refactorisation count
    // exceed the measured cost of a refactorisation
    if (c->prec_fresh) {
      c->prec_base = its;
      c->prec_extra = 0;
      c->prec_fresh = false;
    } else {
      c->prec_extra += std::max(0, its - c->prec_base);
      if (c->prec_extra > c->prec_cost_its) c->prec_valid = false;
    }
    tt = c->timer_begin(TM_BACKSUB);
    HTRY(launch_backsub(c, dx, U, part));
    hipLaunchKernelGGL(facet_update_kernel, dim3(fb), dim3(256), 0, c->stream, n, dx, Uhat, part + 2 * c->n_im);
    c->timer_end(tt);
    HTRY(hipGetLastError());
    // the four norms into coherent host memory; the host spins on the last one (>= 0 or
    // infinite, never the sentinel -1)
    double* hn = w.hgm + GM_MAXM + 2;
    hn[3] = -1.0;
    hipLaunchKernelGGL(newton_norms_kernel, dim3(1), dim3(256), 0, c->stream, c->n_im, fb, part,
                       w.hgm_dev + GM_MAXM + 2);
    HTRY(hipGetLastError());
    HTRY(wait_host_value(c, &hn[3], -1.0));
    c->timers_resolve();
    const double du = hn[0], uu = hn[1], dh = hn[2], hh = hn[3];
    if (!std::isfinite(du) || !std::isfinite(dh) || !std::isfinite(uu) || !std::isfinite(hh)) {
      c->err = "non-finite Newton increment";
      return IMEX_ENONFINITE;
    }
    last = (uu > 0.0) ? du / uu : du;
    dz_prev = std::fmax(last, hh > 0.0 ? dh / hh : dh);
    if (st && st->n_hist < (int)(sizeof(st->du_hist) / sizeof(double))) st->du_hist[st->n_hist++] = dz_prev;
    const double tu = c->opt.newton_rtol * uu, th = c->opt.newton_rtol * hh;
    // a correction whose facet solve stopped at gmres_maxit short of its tolerance
    // certifies nothing (a stalled solve gives a small increment): iterate on
    if (!gm_reached) {
      ++gm_capped;
      q_last = SIMPLIFIED_QMAX;             // the next correction assembles a Jacobian
      du_prev = 0.0;
      dh_prev = 0.0;
      continue;
    }
    if (du <= tu && dh <= th) { converged = true; break; }
    if (it >= 2 && du_prev > 0.0 && dh_prev > 0.0) {
      const double qu = du / du_prev, qh = dh / dh_prev;
      q_last = std::fmax(qu, qh);
      if (it == 2) q2 = q_last;
      if (qu < 0.5 && qh < 0.5 && qu / (1.0 - qu) * du <= tu && qh / (1.0 - qh) * dh <= th) {
        converged = true;
        break;
      }
    } else {
      // no contraction measured yet: a chord step may follow the first Jacobian
      q_last = 0.0;
    }
    du_prev = du;
    dh_prev = dh;
  }
  if (q2 > 0.0) c->newton_q2 = q2;
  if (st) {
    st->newton_its = newton;
    st->gmres_its = gm_total;
    st->newton_last_du = last;
    st->n_jacobians = nfull;
  }
  // R^HDG and the mixed variables at the converged state.  Also after a simplified
  // correction: the contraction test accepts increments up to about rtol / theta, and
  // R^HDG feeds the later stages' right-hand sides through the stiff (K - M) / dt_a.
  HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 0, R_out));
  HTRY(hipStreamSynchronize(c->stream));
  if (!converged) {
    c->err = "Newton did not converge within newton_maxit";
    if (gm_capped) c->err += " (" + std::to_string(gm_capped) + " facet solves stopped at gmres_maxit)";
    return IMEX_ENOCONV;
  }
  return IMEX_OK;
}

// Reverse mode of one implicit stage at its converged state (Y: stage state, explicit rows
// holding the interface data y^ex_{i+1}; H: facet state).  Given the adjoint Rhbar of
// R^HDG_i (element rows) and the adjoints ybar (implicit rows of y^im_i, in/out) and hbar
// (Uhat_i, in/out) it
//   1. adds the transposed Jacobian of R^HDG: ybar += (K - M)^T Rhbar / dt_a,
//      hbar += C^T Rhbar / dt_a;
//   2. solves J^T [lam; lamhat] = [ybar; hbar] (condensed, GMRES on S^T with a facet
//      block-Jacobi preconditioner);
//   3. returns rhsbar = lam (the stage equation is M y + dt_a R - rhs = 0) and adds the
//      adjoint of the interface data to yexbar (explicit rows).
imex_status hdg_stage_adjoint(imex_ctx* c, double dt_a, const double* Y, const double* H, const double* Rhbar,
                              double* ybar, double* hbar, double* rhsbar, double* yexbar, int* gmres_its) {
  Workspace& w = c->ws;
  const int nh = c->n_hf * 4 * c->NP;
  if (!w.adj_P) {
    const size_t NFF = 4 * c->NP;
    HTRY(hipMalloc(&w.adj_P, 8 * (size_t)c->n_hf * NFF * NFF));
    HTRY(hipMalloc(&w.adj_w, 8 * (size_t)c->E * 4 * c->NN));
    w.bytes += 8 * ((size_t)c->n_hf * NFF * NFF + (size_t)c->E * 4 * c->NN);
  }
  HTRY(launch_assemble(c, dt_a, Y, H, nullptr, 1, nullptr));
  HTRY(launch_condense(c));
  const int m = c->opt.gmres_restart;
  double* b = w.gm + (size_t)nh * (m + 3);
  double* lh = b + nh;
  HDG_DISPATCH_ST(c->K, LA_DISPATCH(c, {
    const LT* blk = la<LT>(w.blk);
    const LT* Kinv = la<LT>(w.Kinv);
    const size_t bs = blk_stride(c);
    const int nfb = (nh + 127) / 128;
    if (Rhbar) {
      hipLaunchKernelGGL((elem_KT_kernel<KK, LT>), dim3(c->n_im), dim3(128), 0, c->stream, c->dmesh(), c->dhdg(), bs,
                         blk, dt_a, Rhbar, ybar);
      // hbar += C^T Rhbar / (dt_a dts_e): the element scale is folded into a scaled copy
      hipLaunchKernelGGL(rows_scale_kernel<KK>, dim3((c->n_im * 4 * c->NN + 255) / 256), dim3(256), 0, c->stream,
                         c->dmesh(), c->dhdg(), dt_a, Rhbar, w.adj_w);
      hipLaunchKernelGGL((facet_CT_kernel<KK, LT>), dim3(nfb), dim3(128), 0, c->stream, c->dhdg(), bs, blk, w.adj_w,
                         1.0, hbar);
    }
    // b = hbar - C^T K^-T ybar
    hipLaunchKernelGGL((kinvT_kernel<KK, LT>), dim3(c->n_im), dim3(128), 0, c->stream, c->dhdg(), Kinv, ybar, w.adj_w);
    HTRY(hipMemcpyAsync(b, hbar, sizeof(double) * nh, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL((facet_CT_kernel<KK, LT>), dim3(nfb), dim3(128), 0, c->stream, c->dhdg(), bs, blk, w.adj_w,
                       -1.0, b);
    hipLaunchKernelGGL((bjT_factor_kernel<KK, LT>), dim3(c->n_hf), dim3(64), 0, c->stream, c->dhdg(), bs, blk, w.adj_P);
  }));
  HTRY(hipGetLastError());
  c->adj_mode = true;
  const double rtol = c->opt.gmres_rtol;
  c->opt.gmres_rtol = std::min(rtol, 1e-12);
  int its = 0;
  bool reached = false;
  imex_status st = gmres(c, b, lh, &its, 5, &reached);
  c->opt.gmres_rtol = rtol;
  c->adj_mode = false;
  if (st != IMEX_OK) return st;
  if (!reached) {
    c->err = "transposed facet solve stopped at gmres_maxit short of its tolerance";
    return IMEX_ENOCONV;
  }
  if (gmres_its) *gmres_its = its;
  HDG_DISPATCH_ST(c->K, LA_DISPATCH(c, {
    hipLaunchKernelGGL((backsubT_kernel<KK, LT>), dim3(c->n_im), dim3(128), 0, c->stream, c->dhdg(), blk_stride(c),
                       la<LT>(w.blk), la<LT>(w.Kinv), ybar, lh, rhsbar);
    hipLaunchKernelGGL(interfaceT_kernel<KK>, dim3((c->E * c->NN + 255) / 256), dim3(256), 0, c->stream, c->dmesh(),
                       c->d_ex_ifacet, lh, yexbar);
  }));
  HTRY(hipGetLastError());
  return IMEX_OK;
}

// R^HDG (implicit rows of Rh) and the facet residual shares (ws.hres) at (Y, H), FP64
hipError_t launch_hdg_residual(imex_ctx* c, double dt_a, const double* Y, const double* H, double* Rh) {
  return launch_assemble(c, dt_a, Y, H, nullptr, 0, Rh);
}

// the facet part of the last hdg_stage_adjoint solution (valid until the next facet solve)
const double* adjoint_facet_solution(const imex_ctx* c) {
  const size_t nh = (size_t)c->n_hf * 4 * c->NP;
  return c->ws.gm + nh * (c->opt.gmres_restart + 3) + nh;
}

// dst[b][i][j] = src[b * sstride + i * sld + j] for b < batch, i < rows, j < cols (dst dense, FP64)
template <class T>
__global__ void copy_blocks_kernel(int batch, int rows, int cols, const T* __restrict__ src, int sld,
                                   long long sstride, double* __restrict__ dst) {
  const long long n = (long long)batch * rows * cols;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
    const long long b = t / ((long long)rows * cols);
    const int r = (int)((t / cols) % rows), j = (int)(t % cols);
    dst[t] = (double)src[b * sstride + (long long)r * sld + j];
  }
}

imex_status hdg_local_system(imex_ctx* c, double dt_a, const double* rhs, const double* U, const double* Uhat,
                             double* f, double* h, double* K, double* C, double* D, double* E) {
  HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 1, nullptr));
  const int NU = 4 * c->NN, NF = 16 * c->NP, NC = NU + NF + 1;
  const long long bs = (long long)blk_stride(c);
  struct Part { int r0, c0, rows, cols; double* dst; };
  const Part parts[5] = {{0, NC - 1, NU, 1, f}, {0, 0, NU, NU, K}, {0, NU, NU, NF, C}, {NU, 0, NF, NU, D},
                         {NU, NU, NF, NF, E}};
  HTRY(hipMemcpyAsync(h, c->ws.hres, sizeof(double) * (size_t)c->n_im * NF, hipMemcpyDeviceToDevice, c->stream));
  for (const Part& pt : parts) {
    LA_DISPATCH(c, {
      const LT* src = la<LT>(c->ws.blk) + (size_t)pt.r0 * NC + pt.c0;
      hipLaunchKernelGGL(copy_blocks_kernel<LT>, dim3(1024), dim3(256), 0, c->stream, c->n_im, pt.rows, pt.cols, src,
                         NC, bs, pt.dst);
    });
    HTRY(hipGetLastError());
  }
  HTRY(hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

}  // namespace imex
