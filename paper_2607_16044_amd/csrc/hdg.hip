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
#include <cmath>
#include <cstring>
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
  static constexpr size_t BLK = (size_t)NU + NF + (size_t)NU * NU + 2 * (size_t)NU * NF + (size_t)NF * NF;
  static constexpr size_t SCR = MX ? (2 * (size_t)NU * NQM + 2 * (size_t)NQM * NF) : 0;
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
struct AsmParams {
  double dt_a;
  double alpha;
  int lf;
  int jacobian;      // 0: residual only
};

template <int K, bool MX> struct AsmShared {
  using S = HS<K, MX>;
  BasisTable tb;
  double U[S::NU];
  double Uh[S::NF];                   // [face][v][m]
  double Q[MX ? S::NQM : 1];          // [c][n]
  double uex[4][S::NQ][4];
  double VV[S::NQV][8];               // volume point outputs
  double JV[S::NQV][8][S::NIV];       // d out / d in at volume points
  double VF[4][S::NQ][S::NOF];        // face point outputs
  double JF[4][S::NQ][S::NOF][S::NIF];
  double PL[S::NQV][3];               // lifting inputs at volume points (MX)
  double JL[MX ? S::NQV : 1][3][4];
  double PLF[4][S::NQ][3];
  double JLF[MX ? 4 : 1][S::NQ][3][4];
  double Gv[S::NQV][8];               // grad U at volume points (IP)
  double Gf[4][S::NQ][8];             // grad U at face points (IP)
  double Wv[S::NQV][4];
  double Wf[4][S::NQ][4];
  double Wh[4][S::NQ][4];
  double Qv[MX ? S::NQV : 1][5];
  double Qf[MX ? 4 : 1][S::NQ][5];
};

template <int K, bool MX>
__global__ void __launch_bounds__(256) hdg_assemble_kernel(DeviceMesh m, DeviceHDG h, Gas g, AsmParams prm,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ Uhat,
                                                           const double* __restrict__ rhs, double* __restrict__ blk,
                                                           double* __restrict__ scr, double* __restrict__ Qout,
                                                           double* __restrict__ Rh) {
  using S = HS<K, MX>;
  constexpr int NP = S::NP, NQ = S::NQ, NN = S::NN, NQV = S::NQV, NU = S::NU, NF = S::NF, NFF = S::NFF;
  constexpr int NQM = S::NQM, NIV = S::NIV, NIF = S::NIF, NOF = S::NOF;
  extern __shared__ double smem_raw[];
  AsmShared<K, MX>& sh = *reinterpret_cast<AsmShared<K, MX>*>(smem_raw);
  const int p = blockIdx.x;
  const int e = h.im_list[p];
  const int tid = threadIdx.x, nt = blockDim.x;
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
  // ---- point-wise outputs and Jacobians (dual numbers, 4 seeds per pass) ----
  constexpr int CV = (NIV + 3) / 4, CF = (NIF + 3) / 4, CL = 1;
  const int ntask = NQV * CV + 4 * NQ * CF + (MX ? (NQV + 4 * NQ) * CL : 0);
  for (int task = tid; task < (prm.jacobian ? ntask : NQV + 4 * NQ); task += nt) {
    if (!prm.jacobian) {
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
    using D4 = Dual<4>;
    if (task < NQV * CV) {
      const int qv = task / CV, ch = task % CV;
      // inputs: 0..3 U, then (MX) 4..8 Q, (IP) 4..11 grad U as [v][d]
      D4 W[4];
      for (int v = 0; v < 4; ++v) {
        W[v] = D4(sh.Wv[qv][v]);
        const int idx = v - 4 * ch;
        if (idx >= 0 && idx < 4) W[v].d[idx] = 1.0;
      }
      D4 out[4][2];
      if (MX) {
        D4 Qd[5];
        for (int c = 0; c < 5; ++c) {
          Qd[c] = D4(sh.Qv[qv][c]);
          const int idx = 4 + c - 4 * ch;
          if (idx >= 0 && idx < 4) Qd[c].d[idx] = 1.0;
        }
        vol_point_mx(W, Qd, g, out);
      } else {
        D4 G[4][2];
        for (int v = 0; v < 4; ++v)
          for (int d = 0; d < 2; ++d) {
            G[v][d] = D4(sh.Gv[qv][2 * v + d]);
            const int idx = 4 + 2 * v + d - 4 * ch;
            if (idx >= 0 && idx < 4) G[v][d].d[idx] = 1.0;
          }
        vol_point_ip(W, G, g, out);
      }
      for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 2; ++d) {
          if (ch == 0) sh.VV[qv][2 * v + d] = out[v][d].v;
          for (int k = 0; k < 4; ++k) {
            const int col = 4 * ch + k;
            if (col < NIV) sh.JV[qv][2 * v + d][col] = out[v][d].d[k];
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
        int idx = v - 4 * ch;
        if (idx >= 0 && idx < 4) W[v].d[idx] = 1.0;
        idx = 4 + v - 4 * ch;
        if (idx >= 0 && idx < 4) Wh[v].d[idx] = 1.0;
      }
      if (MX) {
        D4 Qd[5], s[4], t[4];
        for (int c = 0; c < 5; ++c) {
          Qd[c] = D4(sh.Qf[f][q][c]);
          const int idx = 8 + c - 4 * ch;
          if (idx >= 0 && idx < 4) Qd[c].d[idx] = 1.0;
        }
        face_point_mx(W, Wh, Qd, fd, g, s, t);
        for (int v = 0; v < 4; ++v) {
          if (ch == 0) { sh.VF[f][q][v] = s[v].v; sh.VF[f][q][4 + v] = t[v].v; }
          for (int k = 0; k < 4; ++k) {
            const int col = 4 * ch + k;
            if (col < NIF) { sh.JF[f][q][v][col] = s[v].d[k]; sh.JF[f][q][4 + v][col] = t[v].d[k]; }
          }
        }
      } else {
        D4 G[4][2], s[4], gc[4][2], t[4];
        for (int v = 0; v < 4; ++v)
          for (int d = 0; d < 2; ++d) {
            G[v][d] = D4(sh.Gf[f][q][2 * v + d]);
            const int idx = 8 + 2 * v + d - 4 * ch;
            if (idx >= 0 && idx < 4) G[v][d].d[idx] = 1.0;
          }
        face_point_ip(W, G, Wh, fd, g, s, gc, t);
        for (int v = 0; v < 4; ++v) {
          if (ch == 0) {
            sh.VF[f][q][v] = s[v].v;
            sh.VF[f][q][4 + 2 * v] = gc[v][0].v;
            sh.VF[f][q][5 + 2 * v] = gc[v][1].v;
            sh.VF[f][q][12 + v] = t[v].v;
          }
          for (int k = 0; k < 4; ++k) {
            const int col = 4 * ch + k;
            if (col < NIF) {
              sh.JF[f][q][v][col] = s[v].d[k];
              sh.JF[f][q][4 + 2 * v][col] = gc[v][0].d[k];
              sh.JF[f][q][5 + 2 * v][col] = gc[v][1].d[k];
              sh.JF[f][q][12 + v][col] = t[v].d[k];
            }
          }
        }
      }
    } else if (MX) {
      const int i = task - NQV * CV - 4 * NQ * CF;
      D4 W[4], P[3];
      const double* src = (i < NQV) ? sh.Wv[i] : sh.Wh[(i - NQV) / NQ][(i - NQV) % NQ];
      for (int v = 0; v < 4; ++v) { W[v] = D4(src[v]); W[v].d[v] = 1.0; }
      lift_point(W, g, P);
      for (int c = 0; c < 3; ++c)
        for (int v = 0; v < 4; ++v) {
          if (i < NQV) sh.JL[i][c][v] = P[c].d[v];
          else sh.JLF[(i - NQV) / NQ][(i - NQV) % NQ][c][v] = P[c].d[v];
        }
    }
  }
  __syncthreads();
  // ---- residual rows ---------------------------------------------------------
  double* bp = blk + (size_t)p * S::BLK;
  double* fr = bp;
  double* hr = bp + NU;
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
      fr[r] = mass * sh.U[r] + prm.dt_a * acc - (rhs ? rhs[gi] : 0.0);
    } else {
      const int rr = r - NU, f = rr / NFF, v = (rr % NFF) / NP, mm = rr % NP;
      const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
      constexpr int TO = MX ? 4 : 12;
      double acc = 0.0;
      for (int q = 0; q < NQ; ++q) acc += tb.W[q] * wl * tb.L[q][mm] * sh.VF[f][q][TO + v];
      hr[rr] = acc;
    }
  }
  if (!prm.jacobian) return;
  // ---- Jacobian blocks ---------------------------------------------------------
  double* Kb = bp + NU + NF;
  double* Cb = Kb + NU * NU;
  double* Db = Cb + NU * NF;
  double* Eb = Db + NF * NU;
  constexpr int TO = MX ? 4 : 12;         // offset of t rows among face outputs
  constexpr int UHI = 4;                  // offset of Uhat among face inputs
  constexpr int XF = 8;                   // offset of (Q | grad U) among face inputs
  // K = M + dt_a dR/dU
  for (int idx = tid; idx < NU * NU; idx += nt) {
    const int row = idx / NU, col = idx % NU;
    const int v = row / NN, n = row % NN, a = n % NP, b = n / NP;
    const int v2 = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
    double acc = 0.0;
    for (int qj = 0; qj < NQ; ++qj)
      for (int qi = 0; qi < NQ; ++qi) {
        const int qv = qi + NQ * qj;
        const double w = tb.W[qi] * tb.W[qj] * jac;
        const double tx = tb.D[qi][a] * tb.L[qj][b] * sx, ty = tb.L[qi][a] * tb.D[qj][b] * sy;
        const double ph2 = tb.L[qi][a2] * tb.L[qj][b2];
        const double* jx = sh.JV[qv][2 * v];
        const double* jy = sh.JV[qv][2 * v + 1];
        double dx = jx[v2] * ph2, dy = jy[v2] * ph2;
        if (!MX) {
          const double px2 = tb.D[qi][a2] * tb.L[qj][b2] * sx, py2 = tb.L[qi][a2] * tb.D[qj][b2] * sy;
          dx += jx[4 + 2 * v2] * px2 + jx[5 + 2 * v2] * py2;
          dy += jy[4 + 2 * v2] * px2 + jy[5 + 2 * v2] * py2;
        }
        acc += w * (tx * dx + ty * dy);
      }
    for (int f = 0; f < 4; ++f) {
      const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
      for (int q = 0; q < NQ; ++q) {
        double ph, pxi, peta, ph2, pxi2, peta2;
        face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
        face_basis<K>(tb, f, q, a2, b2, ph2, pxi2, peta2);
        const double w = tb.W[q] * wl;
        const double* js = sh.JF[f][q][v];
        double d = js[v2] * ph2;
        if (!MX) {
          d += js[XF + 2 * v2] * pxi2 * sx + js[XF + 1 + 2 * v2] * peta2 * sy;
          const double* jgx = sh.JF[f][q][4 + 2 * v];
          const double* jgy = sh.JF[f][q][5 + 2 * v];
          const double dgx = jgx[v2] * ph2 + jgx[XF + 2 * v2] * pxi2 * sx + jgx[XF + 1 + 2 * v2] * peta2 * sy;
          const double dgy = jgy[v2] * ph2 + jgy[XF + 2 * v2] * pxi2 * sx + jgy[XF + 1 + 2 * v2] * peta2 * sy;
          acc += w * (pxi * sx * dgx + peta * sy * dgy);
        }
        acc += w * ph * d;
      }
    }
    Kb[idx] = prm.dt_a * acc + ((row == col) ? tb.NW[a] * tb.NW[b] * jac : 0.0);
  }
  // C = dt_a dR/dUhat (each column lives on one face)
  for (int idx = tid; idx < NU * NF; idx += nt) {
    const int row = idx / NF, col = idx % NF;
    const int v = row / NN, n = row % NN, a = n % NP, b = n / NP;
    const int f = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP;
    const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
    double acc = 0.0;
    for (int q = 0; q < NQ; ++q) {
      double ph, pxi, peta;
      face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
      const double w = tb.W[q] * wl * tb.L[q][m2];
      acc += w * ph * sh.JF[f][q][v][UHI + v2];
      if (!MX) acc += w * (pxi * sx * sh.JF[f][q][4 + 2 * v][UHI + v2] + peta * sy * sh.JF[f][q][5 + 2 * v][UHI + v2]);
    }
    Cb[idx] = prm.dt_a * acc;
  }
  // D = dh/dU, E = dh/dUhat (E block-diagonal over faces before the mixed elimination)
  for (int idx = tid; idx < NF * NU; idx += nt) {
    const int row = idx / NU, col = idx % NU;
    const int f = row / NFF, v = (row % NFF) / NP, mm = row % NP;
    const int v2 = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
    const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
    double acc = 0.0;
    for (int q = 0; q < NQ; ++q) {
      double ph2, pxi2, peta2;
      face_basis<K>(tb, f, q, a2, b2, ph2, pxi2, peta2);
      const double* jt = sh.JF[f][q][TO + v];
      double d = jt[v2] * ph2;
      if (!MX) d += jt[XF + 2 * v2] * pxi2 * sx + jt[XF + 1 + 2 * v2] * peta2 * sy;
      acc += tb.W[q] * wl * tb.L[q][mm] * d;
    }
    Db[idx] = acc;
  }
  for (int idx = tid; idx < NF * NF; idx += nt) {
    const int row = idx / NF, col = idx % NF;
    const int f = row / NFF, v = (row % NFF) / NP, mm = row % NP;
    const int f2 = col / NFF, v2 = (col % NFF) / NP, m2 = col % NP;
    double acc = 0.0;
    if (f == f2) {
      const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
      for (int q = 0; q < NQ; ++q)
        acc += tb.W[q] * wl * tb.L[q][mm] * tb.L[q][m2] * sh.JF[f][q][TO + v][UHI + v2];
    }
    Eb[idx] = acc;
  }
  if (MX) {
    // mixed blocks: A12 = dt_a dR/dQ, A32 = dh/dQ, A21 = dg/dU, A23 = dg/dUhat (g = M_Q Q + l)
    double* A12 = scr + (size_t)p * S::SCR;
    double* A21 = A12 + NU * NQM;
    double* A23 = A21 + NQM * NU;
    double* A32 = A23 + NQM * NF;
    for (int idx = tid; idx < NU * NQM; idx += nt) {
      const int row = idx / NQM, col = idx % NQM;
      const int v = row / NN, n = row % NN, a = n % NP, b = n / NP;
      const int c = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
      double acc = 0.0;
      for (int qj = 0; qj < NQ; ++qj)
        for (int qi = 0; qi < NQ; ++qi) {
          const int qv = qi + NQ * qj;
          const double w = tb.W[qi] * tb.W[qj] * jac;
          const double tx = tb.D[qi][a] * tb.L[qj][b] * sx, ty = tb.L[qi][a] * tb.D[qj][b] * sy;
          const double ph2 = tb.L[qi][a2] * tb.L[qj][b2];
          acc += w * ph2 * (tx * sh.JV[qv][2 * v][4 + c] + ty * sh.JV[qv][2 * v + 1][4 + c]);
        }
      for (int f = 0; f < 4; ++f) {
        const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
        for (int q = 0; q < NQ; ++q) {
          double ph, pxi, peta, ph2, pxi2, peta2;
          face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
          face_basis<K>(tb, f, q, a2, b2, ph2, pxi2, peta2);
          acc += tb.W[q] * wl * ph * ph2 * sh.JF[f][q][v][XF + c];
        }
      }
      A12[idx] = prm.dt_a * acc;
    }
    for (int idx = tid; idx < NF * NQM; idx += nt) {
      const int row = idx / NQM, col = idx % NQM;
      const int f = row / NFF, v = (row % NFF) / NP, mm = row % NP;
      const int c = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
      const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
      double acc = 0.0;
      for (int q = 0; q < NQ; ++q) {
        double ph2, pxi2, peta2;
        face_basis<K>(tb, f, q, a2, b2, ph2, pxi2, peta2);
        acc += tb.W[q] * wl * tb.L[q][mm] * ph2 * sh.JF[f][q][TO + v][XF + c];
      }
      A32[idx] = acc;
    }
    // lifting coefficients: l_c[n] = sum_q w sum_p cvol(c,p,d) P_p dphi_n/dx_d - sum_f,q w phi_n sum_p cfac(c,p,n) P_p
    for (int idx = tid; idx < NQM * (NU + NF); idx += nt) {
      const int row = idx / (NU + NF), col = idx % (NU + NF);
      const int c = row / NN, n = row % NN, a = n % NP, b = n / NP;
      double acc = 0.0;
      if (col < NU) {
        const int v2 = col / NN, n2 = col % NN, a2 = n2 % NP, b2 = n2 / NP;
        for (int qj = 0; qj < NQ; ++qj)
          for (int qi = 0; qi < NQ; ++qi) {
            const int qv = qi + NQ * qj;
            const double w = tb.W[qi] * tb.W[qj] * jac * tb.L[qi][a2] * tb.L[qj][b2];
            const double px = tb.D[qi][a] * tb.L[qj][b] * sx, py = tb.L[qi][a] * tb.D[qj][b] * sy;
            const double du = sh.JL[qv][0][v2], dv = sh.JL[qv][1][v2], dth = sh.JL[qv][2][v2];
            double d;
            switch (c) {
              case 0: d = (2.0 / 3.0) * du * px - (1.0 / 3.0) * dv * py; break;
              case 1: d = du * py + dv * px; break;
              case 2: d = -(1.0 / 3.0) * du * px + (2.0 / 3.0) * dv * py; break;
              case 3: d = dth * px; break;
              default: d = dth * py; break;
            }
            acc += w * d;
          }
        A21[(size_t)row * NU + col] = acc;
      } else {
        const int cc = col - NU;
        const int f = cc / NFF, v2 = (cc % NFF) / NP, m2 = cc % NP;
        double nx, ny;
        fnormal(f, nx, ny);
        const double wl = (f < 2) ? 0.5 * hy : 0.5 * hx;
        for (int q = 0; q < NQ; ++q) {
          double ph, pxi, peta;
          face_basis<K>(tb, f, q, a, b, ph, pxi, peta);
          const double w = tb.W[q] * wl * ph * tb.L[q][m2];
          const double du = sh.JLF[f][q][0][v2], dv = sh.JLF[f][q][1][v2], dth = sh.JLF[f][q][2][v2];
          double d;
          switch (c) {
            case 0: d = (2.0 / 3.0) * du * nx - (1.0 / 3.0) * dv * ny; break;
            case 1: d = du * ny + dv * nx; break;
            case 2: d = -(1.0 / 3.0) * du * nx + (2.0 / 3.0) * dv * ny; break;
            case 3: d = dth * nx; break;
            default: d = dth * ny; break;
          }
          acc -= w * d;
        }
        A23[(size_t)row * NF + cc] = acc;
      }
    }
  }
}

// HDG-MX: eliminate the mixed block, A22 = M_Q diagonal:
//   K -= A12 A22^-1 A21, C -= A12 A22^-1 A23, D -= A32 A22^-1 A21, E -= A32 A22^-1 A23
template <int K>
__global__ void __launch_bounds__(256) hdg_eliminate_kernel(DeviceMesh m, DeviceHDG h, double* __restrict__ blk,
                                                            const double* __restrict__ scr) {
  using S = HS<K, true>;
  constexpr int NP = S::NP, NN = S::NN, NU = S::NU, NF = S::NF, NQM = S::NQM;
  __shared__ double minv[NQM];
  const int p = blockIdx.x;
  const int e = h.im_list[p];
  const BasisTable& tb = *m.tab;
  const double jac = 0.25 * m.hx[e] * m.hy[e];
  for (int i = threadIdx.x; i < NQM; i += blockDim.x) {
    const int c = i / NN, n = i % NN;
    minv[i] = 1.0 / ((c == 1 ? 2.0 : 1.0) * tb.NW[n % NP] * tb.NW[n / NP] * jac);
  }
  __syncthreads();
  const double* A12 = scr + (size_t)p * S::SCR;
  const double* A21 = A12 + NU * NQM;
  const double* A23 = A21 + NQM * NU;
  const double* A32 = A23 + NQM * NF;
  double* bp = blk + (size_t)p * S::BLK;
  double* Kb = bp + NU + NF;
  double* Cb = Kb + NU * NU;
  double* Db = Cb + NU * NF;
  double* Eb = Db + NF * NU;
  constexpr int NR = NU + NF;     // rows: K/C rows then D/E rows
  constexpr int NC = NU + NF;     // cols: K/D cols then C/E cols
  for (int idx = threadIdx.x; idx < NR * NC; idx += blockDim.x) {
    const int row = idx / NC, col = idx % NC;
    const double* Lr = (row < NU) ? A12 + (size_t)row * NQM : A32 + (size_t)(row - NU) * NQM;
    double acc = 0.0;
    if (col < NU) {
      for (int k = 0; k < NQM; ++k) acc += Lr[k] * minv[k] * A21[(size_t)k * NU + col];
    } else {
      for (int k = 0; k < NQM; ++k) acc += Lr[k] * minv[k] * A23[(size_t)k * NF + (col - NU)];
    }
    if (row < NU) {
      if (col < NU) Kb[row * NU + col] -= acc;
      else Cb[row * NF + (col - NU)] -= acc;
    } else {
      if (col < NU) Db[(row - NU) * NU + col] -= acc;
      else Eb[(row - NU) * NF + (col - NU)] -= acc;
    }
  }
}

// ---------------------------------------------------------------------------
// condensation: LU of K in LDS, X = K^-1 C, y = K^-1 f, S_T = E - D X, r_T = D y
// ---------------------------------------------------------------------------
template <int K>
__global__ void __launch_bounds__(256) hdg_condense_kernel(DeviceHDG h, size_t blk_stride,
                                                           const double* __restrict__ blk, double* __restrict__ X,
                                                           double* __restrict__ y, double* __restrict__ S,
                                                           double* __restrict__ r, int* __restrict__ info) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP;
  constexpr int CH = 16;                  // right-hand sides per chunk
  extern __shared__ double sm[];
  double* A = sm;                         // NU x NU
  double* B = A + NU * NU;                // NU x CH
  __shared__ int piv[NU];
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  const int p = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* bp = blk + (size_t)p * blk_stride;
  const double* f = bp;
  const double* Kb = bp + NU + NF;
  const double* Cb = Kb + NU * NU;
  const double* Db = Cb + NU * NF;
  const double* Eb = Db + NF * NU;
  for (int i = tid; i < NU * NU; i += nt) A[i] = Kb[i];
  __syncthreads();
  // right-looking LU with partial pivoting
  for (int j = 0; j < NU; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < NU; i += nt) {
      const double v = fabs(A[i * NU + j]);
      if (v > best) { best = v; bi = i; }
    }
    red_v[tid] = best;
    red_i[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s && red_v[tid + s] > red_v[tid]) { red_v[tid] = red_v[tid + s]; red_i[tid] = red_i[tid + s]; }
      __syncthreads();
    }
    const int pr = red_i[0];
    if (tid == 0) {
      piv[j] = pr;
      if (!(red_v[0] > 0.0) && info) info[p] = j + 1;
    }
    if (pr != j)
      for (int c = tid; c < NU; c += nt) {
        const double t = A[j * NU + c];
        A[j * NU + c] = A[pr * NU + c];
        A[pr * NU + c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[j * NU + j];
    for (int i = j + 1 + tid; i < NU; i += nt) A[i * NU + j] *= inv;
    __syncthreads();
    const int rem = NU - j - 1;
    for (int idx = tid; idx < rem * rem; idx += nt) {
      const int i = j + 1 + idx / rem, c = j + 1 + idx % rem;
      A[i * NU + c] -= A[i * NU + j] * A[j * NU + c];
    }
    __syncthreads();
  }
  // solve for [f | C] in chunks of CH columns
  constexpr int NRHS = 1 + NF;
  double* Xp = X + (size_t)p * NU * NF;
  double* yp = y + (size_t)p * NU;
  for (int c0 = 0; c0 < NRHS; c0 += CH) {
    const int nc = (NRHS - c0 < CH) ? NRHS - c0 : CH;
    for (int idx = tid; idx < NU * CH; idx += nt) {
      const int i = idx / CH, c = idx % CH;
      const int col = c0 + c;
      double v = 0.0;
      if (c < nc) v = (col == 0) ? f[i] : Cb[i * NF + (col - 1)];
      B[i * CH + c] = v;
    }
    __syncthreads();
    if (tid < CH) {
      for (int j = 0; j < NU; ++j) {
        const int pr = piv[j];
        if (pr != j) {
          const double t = B[j * CH + tid];
          B[j * CH + tid] = B[pr * CH + tid];
          B[pr * CH + tid] = t;
        }
      }
    }
    __syncthreads();
    for (int j = 0; j < NU; ++j) {            // forward, unit lower
      for (int idx = tid; idx < (NU - j - 1) * CH; idx += nt) {
        const int i = j + 1 + idx / CH, c = idx % CH;
        B[i * CH + c] -= A[i * NU + j] * B[j * CH + c];
      }
      __syncthreads();
    }
    for (int j = NU - 1; j >= 0; --j) {       // backward
      if (tid < CH) B[j * CH + tid] /= A[j * NU + j];
      __syncthreads();
      for (int idx = tid; idx < j * CH; idx += nt) {
        const int i = idx / CH, c = idx % CH;
        B[i * CH + c] -= A[i * NU + j] * B[j * CH + c];
      }
      __syncthreads();
    }
    for (int idx = tid; idx < NU * nc; idx += nt) {
      const int i = idx / nc, c = idx % nc;
      const int col = c0 + c;
      if (col == 0) yp[i] = B[i * CH + c];
      else Xp[i * NF + (col - 1)] = B[i * CH + c];
    }
    __syncthreads();
  }
  // S_T = E - D X, r_T = D y
  __threadfence_block();
  double* Sp = S + (size_t)p * NF * NF;
  double* rp = r + (size_t)p * NF;
  for (int idx = tid; idx < NF * (NF + 1); idx += nt) {
    const int row = idx / (NF + 1), col = idx % (NF + 1);
    double acc = 0.0;
    if (col < NF) {
      for (int k = 0; k < NU; ++k) acc += Db[row * NU + k] * Xp[k * NF + col];
      Sp[row * NF + col] = Eb[row * NF + col] - acc;
    } else {
      for (int k = 0; k < NU; ++k) acc += Db[row * NU + k] * yp[k];
      rp[row] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// facet system
// ---------------------------------------------------------------------------
// b_F = -h_F + sum_T r_T|_F  and the block-Jacobi blocks P_F = sum_T S_T[F, F]
template <int K>
__global__ void facet_rhs_kernel(DeviceHDG h, size_t blk_stride, const double* __restrict__ blk,
                                 const double* __restrict__ r, const double* __restrict__ S, double* __restrict__ b,
                                 double* __restrict__ P) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * NFF) return;
  const int hf = t / NFF, row = t % NFF;
  double acc = 0.0;
  double prow[NFF];
  for (int c = 0; c < NFF; ++c) prow[c] = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * hf + s];
    if (pe < 0) continue;
    const int f = h.hf_face[2 * hf + s];
    const int lr = f * NFF + row;
    acc += -blk[(size_t)pe * blk_stride + NU + lr] + r[(size_t)pe * NF + lr];
    const double* Sr = S + (size_t)pe * NF * NF + (size_t)lr * NF + f * NFF;
    for (int c = 0; c < NFF; ++c) prow[c] += Sr[c];
  }
  b[t] = acc;
  for (int c = 0; c < NFF; ++c) P[((size_t)hf * NFF + row) * NFF + c] = prow[c];
}

// in-place inversion of the per-facet blocks by Gauss-Jordan with partial pivoting
template <int K>
__global__ void __launch_bounds__(64) facet_invert_kernel(int n_hf, double* __restrict__ P, int* __restrict__ info) {
  constexpr int NFF = 4 * (K + 1);
  __shared__ double A[NFF][2 * NFF];
  const int hf = blockIdx.x;
  const int tid = threadIdx.x;
  double* Pp = P + (size_t)hf * NFF * NFF;
  for (int i = tid; i < NFF * 2 * NFF; i += blockDim.x) {
    const int r = i / (2 * NFF), c = i % (2 * NFF);
    A[r][c] = (c < NFF) ? Pp[r * NFF + c] : ((c - NFF == r) ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < NFF; ++j) {
    __shared__ int pr;
    if (tid == 0) {
      int best = j;
      double bv = fabs(A[j][j]);
      for (int i = j + 1; i < NFF; ++i)
        if (fabs(A[i][j]) > bv) { bv = fabs(A[i][j]); best = i; }
      pr = best;
      if (!(bv > 0.0) && info) *info = hf + 1;
    }
    __syncthreads();
    if (pr != j)
      for (int c = tid; c < 2 * NFF; c += blockDim.x) {
        const double t = A[j][c];
        A[j][c] = A[pr][c];
        A[pr][c] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[j][j];
    __syncthreads();
    for (int c = tid; c < 2 * NFF; c += blockDim.x) A[j][c] *= inv;
    __syncthreads();
    for (int idx = tid; idx < NFF * 2 * NFF; idx += blockDim.x) {
      const int i = idx / (2 * NFF), c = idx % (2 * NFF);
      if (i != j) {
        const double fct = A[i][j];
        if (c != j) A[i][c] -= fct * A[j][c];
      }
    }
    __syncthreads();
    for (int i = tid; i < NFF; i += blockDim.x)
      if (i != j) A[i][j] = 0.0;
    __syncthreads();
  }
  for (int i = tid; i < NFF * NFF; i += blockDim.x) Pp[i] = A[i / NFF][NFF + i % NFF];
}

// y = P^-1 x (block diagonal)
template <int K>
__global__ void facet_precond_kernel(int n_hf, const double* __restrict__ Pinv, const double* __restrict__ x,
                                     double* __restrict__ y) {
  constexpr int NFF = 4 * (K + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_hf * NFF) return;
  const int hf = t / NFF, row = t % NFF;
  const double* Pr = Pinv + ((size_t)hf * NFF + row) * NFF;
  const double* xf = x + (size_t)hf * NFF;
  double acc = 0.0;
  for (int c = 0; c < NFF; ++c) acc += Pr[c] * xf[c];
  y[t] = acc;
}

// y = S x, S = sum_T scatter(S_T): each facet row pulls from its adjacent elements
template <int K>
__global__ void facet_apply_kernel(DeviceHDG h, const double* __restrict__ S, const double* __restrict__ x,
                                   double* __restrict__ y) {
  constexpr int NP = K + 1, NF = 16 * NP, NFF = 4 * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= h.n_hf * NFF) return;
  const int hf = t / NFF, row = t % NFF;
  double acc = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int pe = h.hf_side[2 * hf + s];
    if (pe < 0) continue;
    const int f = h.hf_face[2 * hf + s];
    const double* Sr = S + (size_t)pe * NF * NF + (size_t)(f * NFF + row) * NF;
    for (int f2 = 0; f2 < 4; ++f2) {
      const double* xf = x + (size_t)h.efacet[4 * pe + f2] * NFF;
      const double* Sc = Sr + f2 * NFF;
      for (int c = 0; c < NFF; ++c) acc += Sc[c] * xf[c];
    }
  }
  y[t] = acc;
}

// partial dot products of w with each of V_0..V_{k-1} (k <= 64): out[block][k]
__global__ void __launch_bounds__(256) multi_dot_kernel(int n, int k, const double* __restrict__ V, size_t ldv,
                                                        const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  for (int j = 0; j < k; ++j) {
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + tid; i < n; i += gridDim.x * blockDim.x)
      acc += V[(size_t)j * ldv + i] * w[i];
    red[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) out[(size_t)blockIdx.x * k + j] = red[0];
    __syncthreads();
  }
}

// sum the partials: res[j] = sum_b out[b][j]
__global__ void reduce_partials_kernel(int nb, int k, const double* __restrict__ part, double* __restrict__ res) {
  const int j = threadIdx.x;
  if (j >= k) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += part[(size_t)b * k + j];
  res[j] = acc;
}

// w -= sum_j c_j V_j, c read from device memory
__global__ void multi_axpy_kernel(int n, int k, const double* __restrict__ V, size_t ldv,
                                  const double* __restrict__ c, double* __restrict__ w, double sign) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += c[j] * V[(size_t)j * ldv + i];
  w[i] += sign * acc;
}

__global__ void scale_vec_kernel(int n, const double* __restrict__ x, double a, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// back-substitution: dU = -y - X dUhat; U += dU on implicit elements; max |dU|, max |U| per block
template <int K>
__global__ void __launch_bounds__(256) hdg_backsub_kernel(DeviceHDG h, const double* __restrict__ X,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ dUh, double* __restrict__ U,
                                                          double* __restrict__ part) {
  constexpr int NP = K + 1, NN = NP * NP, NU = 4 * NN, NF = 16 * NP, NFF = 4 * NP;
  __shared__ double xs[NF];
  __shared__ double rd[2][256];
  const int p = blockIdx.x;
  const int e = h.im_list[p];
  const int tid = threadIdx.x;
  for (int i = tid; i < NF; i += blockDim.x) xs[i] = dUh[(size_t)h.efacet[4 * p + i / NFF] * NFF + i % NFF];
  __syncthreads();
  double mdu = 0.0, mu = 0.0;
  for (int i = tid; i < NU; i += blockDim.x) {
    const double* Xr = X + ((size_t)p * NU + i) * NF;
    double acc = y[(size_t)p * NU + i];
    for (int c = 0; c < NF; ++c) acc += Xr[c] * xs[c];
    const double du = -acc;
    const double un = U[(size_t)e * NU + i] + du;
    U[(size_t)e * NU + i] = un;
    mdu = fmax(mdu, fabs(du));
    mu = fmax(mu, fabs(un));
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

// Uhat += dUhat; per-block max |dUhat|, max |Uhat|
__global__ void __launch_bounds__(256) facet_update_kernel(int n, const double* __restrict__ d, double* __restrict__ x,
                                                           double* __restrict__ part) {
  __shared__ double rd[2][256];
  const int tid = threadIdx.x;
  double md = 0.0, mx = 0.0;
  for (int i = blockIdx.x * blockDim.x + tid; i < n; i += gridDim.x * blockDim.x) {
    const double xn = x[i] + d[i];
    x[i] = xn;
    md = fmax(md, fabs(d[i]));
    mx = fmax(mx, fabs(xn));
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

static size_t blk_stride(const imex_ctx* c) {
  const size_t NU = 4 * c->NN, NF = 16 * c->NP;
  return NU + NF + NU * NU + 2 * NU * NF + NF * NF;
}
static size_t scr_stride(const imex_ctx* c) {
  if (!use_mx(c)) return 0;
  const size_t NU = 4 * c->NN, NF = 16 * c->NP, NQM = 5 * c->NN;
  return 2 * NU * NQM + 2 * NQM * NF;
}

constexpr int GM_BLOCKS = 64;

size_t hdg_workspace_bytes(const imex_ctx* c) {
  const size_t n_im = c->n_im, NU = 4 * c->NN, NF = 16 * c->NP, NFF = 4 * c->NP, n = (size_t)c->n_hf * NFF;
  const int m = c->opt.gmres_restart;
  return 8 * (n_im * (blk_stride(c) + scr_stride(c) + NU * NF + NU + NF * NF + NF) + (size_t)c->n_hf * NFF * NFF +
              n * (size_t)(m + 6) + (size_t)GM_BLOCKS * (m + 2) + 4 * (size_t)(m + 2) + 2 * (n_im + 1024));
}

imex_status hdg_alloc(imex_ctx* c) {
  if (c->n_im == 0) return IMEX_OK;
  Workspace& w = c->ws;
  const size_t n_im = c->n_im, NU = 4 * c->NN, NF = 16 * c->NP, NFF = 4 * c->NP;
  const size_t n = (size_t)c->n_hf * NFF;
  const int m = c->opt.gmres_restart;
  hipError_t e = hipMalloc(&w.blk, 8 * n_im * blk_stride(c));
  if (e == hipSuccess && scr_stride(c)) e = hipMalloc(&w.scr, 8 * n_im * scr_stride(c));
  if (e == hipSuccess) e = hipMalloc(&w.X, 8 * n_im * NU * NF);
  if (e == hipSuccess) e = hipMalloc(&w.y, 8 * n_im * NU);
  if (e == hipSuccess) e = hipMalloc(&w.S, 8 * n_im * NF * NF);
  if (e == hipSuccess) e = hipMalloc(&w.r, 8 * n_im * NF);
  if (e == hipSuccess) e = hipMalloc(&w.Pinv, 8 * (size_t)c->n_hf * NFF * NFF);
  if (e == hipSuccess) e = hipMalloc(&w.gm, 8 * n * (size_t)(m + 6));
  if (e == hipSuccess) e = hipMalloc(&w.red, 8 * ((size_t)GM_BLOCKS * (m + 2) + 4 * (size_t)(m + 2) + 2 * (n_im + 1024)) + 64);
  if (e == hipSuccess) e = hipHostMalloc(&w.hred, 8 * (4 * (size_t)(m + 2) + 2 * (n_im + 1024)), 0);
  if (e != hipSuccess) {
    c->err = std::string("implicit workspace: ") + hipGetErrorString(e);
    return IMEX_ENOMEM;
  }
  w.bytes += hdg_workspace_bytes(c);
  return IMEX_OK;
}

static hipError_t launch_assemble(imex_ctx* c, double dt_a, const double* U, const double* Uhat, const double* rhs,
                                  int jacobian, double* Rh) {
  AsmParams prm{dt_a, c->opt.alpha_hdg, c->opt.hdg_flux == IMEX_HDG_FLUX_LF, jacobian};
  const bool mx = use_mx(c);
  Workspace& w = c->ws;
  HDG_DISPATCH(c->K, {
    const int ta = jacobian ? c->timer_begin(TM_ASSEMBLE) : -1;
    if (mx) {
      const size_t shm = sizeof(AsmShared<KK, true>);
      hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, true>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, true>), dim3(c->n_im), dim3(256), shm, c->stream, c->dmesh(),
                         c->dhdg(), c->gas, prm, U, Uhat, rhs, w.blk, w.scr, w.Q, Rh);
      c->timer_end(ta);
      if (jacobian) {
        const int te = c->timer_begin(TM_ELIMINATE);
        hipLaunchKernelGGL(hdg_eliminate_kernel<KK>, dim3(c->n_im), dim3(256), 0, c->stream, c->dmesh(), c->dhdg(),
                           w.blk, w.scr);
        c->timer_end(te);
      }
    } else {
      const size_t shm = sizeof(AsmShared<KK, false>);
      hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_assemble_kernel<KK, false>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      hipLaunchKernelGGL((hdg_assemble_kernel<KK, false>), dim3(c->n_im), dim3(256), shm, c->stream, c->dmesh(),
                         c->dhdg(), c->gas, prm, U, Uhat, rhs, w.blk, w.scr, nullptr, Rh);
      c->timer_end(ta);
    }
  });
  return hipGetLastError();
}

static hipError_t launch_condense(imex_ctx* c) {
  Workspace& w = c->ws;
  HDG_DISPATCH(c->K, {
    constexpr int NU = 4 * (KK + 1) * (KK + 1);
    const size_t shm = sizeof(double) * ((size_t)NU * NU + (size_t)NU * 16);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&hdg_condense_kernel<KK>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(hdg_condense_kernel<KK>, dim3(c->n_im), dim3(256), shm, c->stream, c->dhdg(), blk_stride(c),
                       w.blk, w.X, w.y, w.S, w.r, nullptr);
  });
  return hipGetLastError();
}

static hipError_t launch_facet_setup(imex_ctx* c, double* b) {
  Workspace& w = c->ws;
  const int n = c->n_hf * 4 * c->NP;
  HDG_DISPATCH(c->K, {
    hipLaunchKernelGGL(facet_rhs_kernel<KK>, dim3((n + 127) / 128), dim3(128), 0, c->stream, c->dhdg(),
                       blk_stride(c), w.blk, w.r, w.S, b, w.Pinv);
    hipLaunchKernelGGL(facet_invert_kernel<KK>, dim3(c->n_hf), dim3(64), 0, c->stream, c->n_hf, w.Pinv, nullptr);
  });
  return hipGetLastError();
}

static hipError_t launch_precond(imex_ctx* c, const double* x, double* y) {
  const int n = c->n_hf * 4 * c->NP;
  HDG_DISPATCH(c->K, hipLaunchKernelGGL(facet_precond_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                        c->n_hf, c->ws.Pinv, x, y));
  return hipGetLastError();
}

static hipError_t launch_apply(imex_ctx* c, const double* x, double* y) {
  const int n = c->n_hf * 4 * c->NP;
  HDG_DISPATCH(c->K, hipLaunchKernelGGL(facet_apply_kernel<KK>, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                                        c->dhdg(), c->ws.S, x, y));
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

// dots[j] = <V_j, w> for j < k, result copied to host (synchronises)
static imex_status dots_to_host(imex_ctx* c, int n, int k, const double* V, size_t ldv, const double* w, double* dev_res,
                                double* host) {
  double* part = c->ws.red;
  hipLaunchKernelGGL(multi_dot_kernel, dim3(GM_BLOCKS), dim3(256), 0, c->stream, n, k, V, ldv, w, part);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(64), 0, c->stream, GM_BLOCKS, k, part, dev_res);
  HTRY(hipGetLastError());
  HTRY(hipMemcpyAsync(host, dev_res, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
  HTRY(hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

// y += a x
__global__ void axpy_kernel(int n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// Right-preconditioned restarted GMRES on S x = b (x starts at 0).  Classical
// Gram-Schmidt with one re-orthogonalisation pass; Givens rotations on the host.
static imex_status gmres(imex_ctx* c, const double* b, double* x, int* its_out) {
  Workspace& w = c->ws;
  const int n = c->n_hf * 4 * c->NP;
  const int m = c->opt.gmres_restart;
  const size_t ldv = n;
  double* V = w.gm;                       // m+1 basis vectors
  double* z = V + ldv * (m + 1);          // work
  double* r = z + ldv;                    // residual
  double* dres = w.red + (size_t)GM_BLOCKS * (m + 2);
  double* hbuf = w.hred;
  const int nb = (n + 255) / 256;
  HTRY(hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), yv(m);
  imex_status st = dots_to_host(c, n, 1, b, ldv, b, dres, hbuf);
  if (st != IMEX_OK) return st;
  const double bnorm = std::sqrt(hbuf[0]);
  *its_out = 0;
  if (bnorm == 0.0) return IMEX_OK;
  const double tol = c->opt.gmres_rtol * bnorm;
  int total = 0;
  HTRY(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  double beta = bnorm;
  while (total < c->opt.gmres_maxit) {
    hipLaunchKernelGGL(scale_vec_kernel, dim3(nb), dim3(256), 0, c->stream, n, r, 1.0 / beta, V);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int j = 0;
    bool done = false;
    while (j < m && total < c->opt.gmres_maxit) {
      double* vj = V + ldv * j;
      double* vn = V + ldv * (j + 1);
      HTRY(launch_precond(c, vj, z));
      HTRY(launch_apply(c, z, vn));
      for (int pass = 0; pass < 2; ++pass) {
        st = dots_to_host(c, n, j + 1, V, ldv, vn, dres, hbuf);
        if (st != IMEX_OK) return st;
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] += hbuf[i];
        hipLaunchKernelGGL(multi_axpy_kernel, dim3(nb), dim3(256), 0, c->stream, n, j + 1, V, ldv, dres, vn, -1.0);
      }
      st = dots_to_host(c, n, 1, vn, ldv, vn, dres, hbuf);
      if (st != IMEX_OK) return st;
      const double hn = std::sqrt(hbuf[0]);
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0) hipLaunchKernelGGL(scale_vec_kernel, dim3(nb), dim3(256), 0, c->stream, n, vn, 1.0 / hn, vn);
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      const double rr = std::sqrt(a * a + bb * bb);
      cs[j] = (rr > 0.0) ? a / rr : 1.0;
      sn[j] = (rr > 0.0) ? bb / rr : 0.0;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++j;
      ++total;
      if (std::fabs(gv[j]) <= tol || hn == 0.0) { done = true; break; }
    }
    // y = H^-1 g; x += P^-1 (V y)
    for (int i = j - 1; i >= 0; --i) {
      double s = gv[i];
      for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * m + k] * yv[k];
      yv[i] = s / H[(size_t)i * m + i];
    }
    HTRY(hipMemcpyAsync(dres, yv.data(), sizeof(double) * j, hipMemcpyHostToDevice, c->stream));
    HTRY(hipMemsetAsync(r, 0, sizeof(double) * n, c->stream));
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(nb), dim3(256), 0, c->stream, n, j, V, ldv, dres, r, 1.0);
    HTRY(launch_precond(c, r, z));
    hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(256), 0, c->stream, n, 1.0, z, x);
    if (done) break;
    // true residual for the restart: r = b - S x
    HTRY(launch_apply(c, x, r));
    hipLaunchKernelGGL(scale_vec_kernel, dim3(nb), dim3(256), 0, c->stream, n, r, -1.0, r);
    hipLaunchKernelGGL(axpy_kernel, dim3(nb), dim3(256), 0, c->stream, n, 1.0, b, r);
    st = dots_to_host(c, n, 1, r, ldv, r, dres, hbuf);
    if (st != IMEX_OK) return st;
    beta = std::sqrt(hbuf[0]);
    if (beta <= tol) break;
  }
  *its_out = total;
  HTRY(hipGetLastError());
  return IMEX_OK;
}

static hipError_t launch_backsub(imex_ctx* c, const double* dx, double* U, double* part) {
  HDG_DISPATCH(c->K, hipLaunchKernelGGL(hdg_backsub_kernel<KK>, dim3(c->n_im), dim3(256), 0, c->stream, c->dhdg(),
                                        c->ws.X, c->ws.y, dx, U, part));
  return hipGetLastError();
}

imex_status hdg_stage_solve(imex_ctx* c, double dt_a, const double* rhs, double* U, double* Uhat, double* R_out,
                            imex_stats* st) {
  Workspace& w = c->ws;
  const int n = c->n_hf * 4 * c->NP;
  const int m = c->opt.gmres_restart;
  double* b = w.gm + (size_t)n * (m + 3);
  double* dx = b + n;
  double* part = w.red + (size_t)GM_BLOCKS * (m + 2) + 4 * (size_t)(m + 2);
  const int fb = 256;
  int newton = 0, gm_total = 0;
  bool converged = false;
  double last = 0.0;
  for (int it = 1; it <= c->opt.newton_maxit; ++it) {
    newton = it;
    HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 1, nullptr));
    int tt = c->timer_begin(TM_CONDENSE);
    HTRY(launch_condense(c));
    c->timer_end(tt);
    tt = c->timer_begin(TM_FACET);
    HTRY(launch_facet_setup(c, b));
    c->timer_end(tt);
    int its = 0;
    tt = c->timer_begin(TM_GMRES);
    imex_status s = gmres(c, b, dx, &its);
    c->timer_end(tt);
    if (s != IMEX_OK) return s;
    gm_total += its;
    tt = c->timer_begin(TM_BACKSUB);
    HTRY(launch_backsub(c, dx, U, part));
    hipLaunchKernelGGL(facet_update_kernel, dim3(fb), dim3(256), 0, c->stream, n, dx, Uhat, part + 2 * c->n_im);
    c->timer_end(tt);
    HTRY(hipGetLastError());
    const size_t np = 2 * ((size_t)c->n_im + fb);
    HTRY(hipMemcpyAsync(w.hred, part, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream));
    HTRY(hipStreamSynchronize(c->stream));
    c->timers_resolve();
    double du = 0.0, uu = 0.0, dh = 0.0, hh = 0.0;
    for (int i = 0; i < c->n_im; ++i) { du = std::fmax(du, w.hred[2 * i]); uu = std::fmax(uu, w.hred[2 * i + 1]); }
    for (int i = 0; i < fb; ++i) {
      dh = std::fmax(dh, w.hred[2 * (c->n_im + i)]);
      hh = std::fmax(hh, w.hred[2 * (c->n_im + i) + 1]);
    }
    if (!std::isfinite(du) || !std::isfinite(dh) || !std::isfinite(uu) || !std::isfinite(hh)) {
      c->err = "non-finite Newton increment";
      return IMEX_ENONFINITE;
    }
    last = (uu > 0.0) ? du / uu : du;
    if (du <= c->opt.newton_rtol * uu && dh <= c->opt.newton_rtol * hh) { converged = true; break; }
  }
  if (st) {
    st->newton_its = newton;
    st->gmres_its = gm_total;
    st->newton_last_du = last;
  }
  // R^HDG and the mixed variables at the converged state
  HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 0, R_out));
  HTRY(hipStreamSynchronize(c->stream));
  if (!converged) {
    c->err = "Newton did not converge within newton_maxit";
    return IMEX_ENOCONV;
  }
  return IMEX_OK;
}

imex_status hdg_local_system(imex_ctx* c, double dt_a, const double* rhs, const double* U, const double* Uhat,
                             double* f, double* h, double* K, double* C, double* D, double* E) {
  HTRY(launch_assemble(c, dt_a, U, Uhat, rhs, 1, nullptr));
  const size_t NU = 4 * c->NN, NF = 16 * c->NP, bs = blk_stride(c);
  for (int p = 0; p < c->n_im; ++p) {
    const double* bp = c->ws.blk + (size_t)p * bs;
    HTRY(hipMemcpyAsync(f + p * NU, bp, 8 * NU, hipMemcpyDeviceToDevice, c->stream));
    HTRY(hipMemcpyAsync(h + p * NF, bp + NU, 8 * NF, hipMemcpyDeviceToDevice, c->stream));
    HTRY(hipMemcpyAsync(K + p * NU * NU, bp + NU + NF, 8 * NU * NU, hipMemcpyDeviceToDevice, c->stream));
    HTRY(hipMemcpyAsync(C + p * NU * NF, bp + NU + NF + NU * NU, 8 * NU * NF, hipMemcpyDeviceToDevice, c->stream));
    HTRY(hipMemcpyAsync(D + p * NF * NU, bp + NU + NF + NU * NU + NU * NF, 8 * NF * NU, hipMemcpyDeviceToDevice,
                        c->stream));
    HTRY(hipMemcpyAsync(E + p * NF * NF, bp + NU + NF + NU * NU + 2 * NU * NF, 8 * NF * NF, hipMemcpyDeviceToDevice,
                        c->stream));
  }
  HTRY(hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

}  // namespace imex
