// Vector-Jacobian product of the explicit DG-IP residual and of the explicit
// ARK step (reverse mode of Sec. 3.3 and Sec. 4.2.2) on gfx950.
//
// Ubar = (dR^DG/dU)^T Rbar, U over all elements (implicit elements enter only
// through their traces on interface faces), in four launches:
//  1. vjp_trace:   face traces of U and Rbar with their reference derivatives
//  2. vjp_face:    per face Gauss point of every element the adjoint of its
//                  trace and physical gradient, gathered from the element's own
//                  face integrand and from the integrand of the neighbour across
//                  the face (no atomics); point-wise Jacobians by dual numbers
//  3. vjp_volume:  the same for the volume flux at the volume Gauss points
//  4. vjp_contract: contraction with the basis and its gradient (transpose of
//                  the interpolation)
// The adjoint seed of a point is the transpose of the residual's quadrature:
// the coefficient s of phi_n receives w Rbar(x_q), the coefficient of
// dphi_n/dx_d receives w (2/h_d) dRbar/dxi_d(x_q).
#include <vector>

#include "ctx.h"
#include "dg_face.h"

namespace imex {

// (val, d/dxi, d/deta) of a nodal field at face point (f, q)
template <int K>
__device__ inline void vjp_face_interp(const BasisTable& T, int f, int q, const double* u, double o[12]) {
  constexpr int NP = K + 1, NN = NP * NP;
  const int s = f & 1;
#pragma unroll
  for (int i = 0; i < 12; ++i) o[i] = 0.0;
  for (int b = 0; b < NP; ++b)
    for (int a = 0; a < NP; ++a) {
      double ph, pxi, peta;
      if (f < 2) {
        ph = T.LE[s][a] * T.L[q][b];
        pxi = T.DE[s][a] * T.L[q][b];
        peta = T.LE[s][a] * T.D[q][b];
      } else {
        ph = T.L[q][a] * T.LE[s][b];
        pxi = T.D[q][a] * T.LE[s][b];
        peta = T.L[q][a] * T.DE[s][b];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = u[v * NN + a + NP * b];
        o[v] += ph * x;
        o[4 + v] += pxi * x;
        o[8 + v] += peta * x;
      }
    }
}

// 1. TU[e][f][q][12], TR[e][f][q][12]; Rbar rows of implicit elements count as 0
template <int K>
__global__ void __launch_bounds__(256) vjp_trace_kernel(DeviceMesh m, const double* __restrict__ U,
                                                        const double* __restrict__ Rb, double* __restrict__ TU,
                                                        double* __restrict__ TR, const double* __restrict__ Q,
                                                        double* __restrict__ TQ) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * 4 * NQ) return;
  const int q = t % NQ, f = (t / NQ) % 4, e = t / (4 * NQ);
  const BasisTable& tb = *m.tab;
  double o[12];
  vjp_face_interp<K>(tb, f, q, U + (size_t)e * 4 * NN, o);
  for (int i = 0; i < 12; ++i) TU[(size_t)t * 12 + i] = o[i];
  if (m.imp[e]) {
    for (int i = 0; i < 12; ++i) TR[(size_t)t * 12 + i] = 0.0;
    if (Q) {                         // HDG-MX: trace of the mixed variables
      const int s = f & 1;
      const double* qe = Q + (size_t)e * 5 * NN;
      for (int c = 0; c < 5; ++c) {
        double acc = 0.0;
        for (int b = 0; b < NP; ++b)
          for (int a = 0; a < NP; ++a)
            acc += ((f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b]) * qe[c * NN + a + NP * b];
        TQ[(size_t)t * 5 + c] = acc;
      }
    }
  } else {
    vjp_face_interp<K>(tb, f, q, Rb + (size_t)e * 4 * NN, o);
    for (int i = 0; i < 12; ++i) TR[(size_t)t * 12 + i] = o[i];
  }
}

__device__ __forceinline__ double lmeasure(double hx, double hy) { return hx * hy / (2.0 * (hx + hy)); }

// adjoint of the inputs X = (trace U, physical gradient G) of one face integrand:
// Xbar_j += sum s_bar . ds/dX_j + gc_bar : dgc/dX_j.  side 0: X is the element's own
// trace (neighbour data fixed); side 1: X is the neighbour's trace, entering as UN and,
// through F^nu(UN, GN) . n, as fnn (own data fixed).
__device__ inline void face_point_adjoint(int side, int kind, const double Uo[4], const double Go[4][2],
                                          const double UN[4], const double GN[4][2], double nx, double ny,
                                          double tau, int lf, const Gas& g, const double sb[4],
                                          const double gb[4][2], double xb[12]) {
  using D4 = Dual<4>;
  const int nchunk = g.viscous ? 3 : 1;
  for (int ch = 0; ch < nchunk; ++ch) {
    D4 Xu[4], Xg[4][2];
    const double* xu = side == 0 ? Uo : UN;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Xu[v] = D4(xu[v]);
      const int idx = v - 4 * ch;
      if (idx >= 0 && idx < 4) Xu[v].d[idx] = 1.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        Xg[v][d] = D4(side == 0 ? Go[v][d] : GN[v][d]);
        const int idx = 4 + 2 * v + d - 4 * ch;
        if (idx >= 0 && idx < 4) Xg[v][d].d[idx] = 1.0;
      }
    D4 A[4], AG[4][2], B[4], fnn[4];
    if (side == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        A[v] = Xu[v];
        AG[v][0] = Xg[v][0];
        AG[v][1] = Xg[v][1];
        B[v] = D4(UN[v]);
      }
      if (g.viscous && kind != DGF_FARFIELD) {
        double Fn[4][2];
        visc_flux(UN, GN, g, Fn);
#pragma unroll
        for (int v = 0; v < 4; ++v) fnn[v] = D4(Fn[v][0] * nx + Fn[v][1] * ny);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) fnn[v] = D4(0.0);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        A[v] = D4(Uo[v]);
        AG[v][0] = D4(Go[v][0]);
        AG[v][1] = D4(Go[v][1]);
        B[v] = Xu[v];
      }
      if (g.viscous) {
        D4 Fn[4][2];
        visc_flux(Xu, Xg, g, Fn);
#pragma unroll
        for (int v = 0; v < 4; ++v) fnn[v] = Fn[v][0] * nx + Fn[v][1] * ny;
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) fnn[v] = D4(0.0);
      }
    }
    D4 s[4], gc[4][2];
    dg_face_point(kind, A, AG, B, fnn, nx, ny, tau, lf, g, s, gc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int col = 4 * ch + k;
      if (col >= 12) break;
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc += sb[v] * s[v].d[k] + gb[v][0] * gc[v][0].d[k] + gb[v][1] * gc[v][1].d[k];
      xb[col] += acc;
    }
  }
}

// side 1 with an HDG-MX implicit element: its viscous flux is F^nu(U, eps, phi) with the
// lifted mixed variables Q = (eps, phi); X = (trace U, trace Q), adjoints to xb[0..3], qb[0..4]
__device__ inline void face_point_adjoint_mx(int kind, const double Uo[4], const double Go[4][2],
                                             const double UN[4], const double QN[5], double nx, double ny,
                                             double tau, int lf, const Gas& g, const double sb[4],
                                             const double gb[4][2], double xb[12], double qb[5]) {
  using D4 = Dual<4>;
  for (int ch = 0; ch < 3; ++ch) {
    D4 Xu[4], Xq[5], A[4], AG[4][2], fnn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Xu[v] = D4(UN[v]);
      const int idx = v - 4 * ch;
      if (idx >= 0 && idx < 4) Xu[v].d[idx] = 1.0;
      A[v] = D4(Uo[v]);
      AG[v][0] = D4(Go[v][0]);
      AG[v][1] = D4(Go[v][1]);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      Xq[c] = D4(QN[c]);
      const int idx = 4 + c - 4 * ch;
      if (idx >= 0 && idx < 4) Xq[c].d[idx] = 1.0;
    }
    D4 Fn[4][2];
    visc_flux_mx(Xu, Xq, Xq + 3, g, Fn);
#pragma unroll
    for (int v = 0; v < 4; ++v) fnn[v] = Fn[v][0] * nx + Fn[v][1] * ny;
    D4 s[4], gc[4][2];
    dg_face_point(kind, A, AG, Xu, fnn, nx, ny, tau, lf, g, s, gc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int col = 4 * ch + k;
      if (col >= 9) break;
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc += sb[v] * s[v].d[k] + gb[v][0] * gc[v][0].d[k] + gb[v][1] * gc[v][1].d[k];
      if (col < 4) xb[col] += acc;
      else qb[col - 4] += acc;
    }
  }
}

// 2. face-point adjoints PF[e][f][q][12]: (trace adjoint 4, physical-gradient adjoint [v][d] 8)
//    and, for HDG-MX implicit elements, PQ[e][f][q][5] (adjoint of the trace of Q)
template <int K>
__global__ void __launch_bounds__(128) vjp_face_kernel(DeviceMesh m, Gas g, int lf, double alpha,
                                                       const double* __restrict__ TU, const double* __restrict__ TR,
                                                       double* __restrict__ PF, const double* __restrict__ TQ,
                                                       double* __restrict__ PQ) {
  constexpr int NQ = (3 * K + 2) / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * 4 * NQ) return;
  const int q = t % NQ, f = (t / NQ) % 4, e = t / (4 * NQ);
  const BasisTable& tb = *m.tab;
  const double hx = m.hx[e], hy = m.hy[e], sx = 2.0 / hx, sy = 2.0 / hy;
  const double* tu = TU + (size_t)t * 12;
  double Uo[4], Go[4][2];
#pragma unroll
  for (int v = 0; v < 4; ++v) { Uo[v] = tu[v]; Go[v][0] = tu[4 + v] * sx; Go[v][1] = tu[8 + v] * sy; }
  const int nb = m.nbr[4 * e + f];
  double UN[4] = {0, 0, 0, 0}, GN[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  double sxn = 0.0, syn = 0.0;
  const double* tun = nullptr;
  if (nb >= 0) {
    sxn = 2.0 / m.hx[nb];
    syn = 2.0 / m.hy[nb];
    tun = TU + (((size_t)nb * 4 + (f ^ 1)) * NQ + q) * 12;
#pragma unroll
    for (int v = 0; v < 4; ++v) { UN[v] = tun[v]; GN[v][0] = tun[4 + v] * sxn; GN[v][1] = tun[8 + v] * syn; }
  }
  double xb[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) xb[i] = 0.0;
  double nx, ny;
  face_normal(f, nx, ny);
  const double le = lmeasure(hx, hy);
  if (!m.imp[e]) {
    // own integrand: e explicit
    const int kind = nb < 0 ? DGF_FARFIELD : (m.imp[nb] ? DGF_INTERFACE : DGF_INTERIOR);
    const double ln = nb >= 0 ? lmeasure(m.hx[nb], m.hy[nb]) : le;
    const double tau = dg_tau(alpha, K, kind, le, ln);
    const double w = tb.W[q] * ((f < 2) ? 0.5 * hy : 0.5 * hx);
    const double* tr = TR + (size_t)t * 12;
    double sb[4], gb[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) { sb[v] = w * tr[v]; gb[v][0] = w * sx * tr[4 + v]; gb[v][1] = w * sy * tr[8 + v]; }
    if (TQ && kind == DGF_INTERFACE) {
      // the HDG-MX neighbour's viscous flux uses its mixed variables (fixed here)
      const double* tq = TQ + (((size_t)nb * 4 + (f ^ 1)) * NQ + q) * 5;
      double Fn[4][2], fnn[4];
      visc_flux_mx(UN, tq, tq + 3, g, Fn);
#pragma unroll
      for (int v = 0; v < 4; ++v) fnn[v] = Fn[v][0] * nx + Fn[v][1] * ny;
      using D4 = Dual<4>;
      const int nchunk = g.viscous ? 3 : 1;
      for (int ch = 0; ch < nchunk; ++ch) {
        D4 A[4], AG[4][2], B[4], FN[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          A[v] = D4(Uo[v]);
          int idx = v - 4 * ch;
          if (idx >= 0 && idx < 4) A[v].d[idx] = 1.0;
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            AG[v][d] = D4(Go[v][d]);
            idx = 4 + 2 * v + d - 4 * ch;
            if (idx >= 0 && idx < 4) AG[v][d].d[idx] = 1.0;
          }
          B[v] = D4(UN[v]);
          FN[v] = D4(fnn[v]);
        }
        D4 so[4], go[4][2];
        dg_face_point(kind, A, AG, B, FN, nx, ny, tau, lf, g, so, go);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int col = 4 * ch + k;
          if (col >= 12) break;
          double acc = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc += sb[v] * so[v].d[k] + gb[v][0] * go[v][0].d[k] + gb[v][1] * go[v][1].d[k];
          xb[col] += acc;
        }
      }
    } else {
      face_point_adjoint(0, kind, Uo, Go, UN, GN, nx, ny, tau, lf, g, sb, gb, xb);
    }
  }
  double qb[5] = {0, 0, 0, 0, 0};
  if (nb >= 0 && !m.imp[nb]) {
    // the explicit neighbour's integrand on the same face, seen from its side
    const int kind = m.imp[e] ? DGF_INTERFACE : DGF_INTERIOR;
    const double hxn = m.hx[nb], hyn = m.hy[nb];
    const double tau = dg_tau(alpha, K, kind, lmeasure(hxn, hyn), le);
    const int fn = f ^ 1;
    const double w = tb.W[q] * ((fn < 2) ? 0.5 * hyn : 0.5 * hxn);
    const double* tr = TR + (((size_t)nb * 4 + fn) * NQ + q) * 12;
    double sb[4], gb[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) { sb[v] = w * tr[v]; gb[v][0] = w * sxn * tr[4 + v]; gb[v][1] = w * syn * tr[8 + v]; }
    // for the neighbour, "own" is its trace, "neighbour" is this element's
    if (TQ && m.imp[e])
      face_point_adjoint_mx(kind, UN, GN, Uo, TQ + (size_t)t * 5, -nx, -ny, tau, lf, g, sb, gb, xb, qb);
    else
      face_point_adjoint(1, kind, UN, GN, Uo, Go, -nx, -ny, tau, lf, g, sb, gb, xb);
  }
  double* out = PF + (size_t)t * 12;
#pragma unroll
  for (int i = 0; i < 12; ++i) out[i] = xb[i];
  if (PQ && m.imp[e])
#pragma unroll
    for (int c = 0; c < 5; ++c) PQ[(size_t)t * 5 + c] = qb[c];
}

// 3. volume-point adjoints PV[e][qv][12] of explicit elements: F = F^nu(U, G) - F^c(U)
template <int K>
__global__ void __launch_bounds__(128) vjp_volume_kernel(DeviceMesh m, Gas g, const double* __restrict__ U,
                                                         const double* __restrict__ Rb, double* __restrict__ PV) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * NQV) return;
  const int qv = t % NQV, e = t / NQV;
  double* out = PV + (size_t)t * 12;
  if (m.imp[e]) {
    for (int i = 0; i < 12; ++i) out[i] = 0.0;
    return;
  }
  const BasisTable& tb = *m.tab;
  const int qi = qv % NQ, qj = qv / NQ;
  const double hx = m.hx[e], hy = m.hy[e], sx = 2.0 / hx, sy = 2.0 / hy;
  const double* ue = U + (size_t)e * 4 * NN;
  const double* re = Rb + (size_t)e * 4 * NN;
  double W[4] = {0, 0, 0, 0}, G[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}}, rx[4] = {0, 0, 0, 0}, ry[4] = {0, 0, 0, 0};
  for (int b = 0; b < NP; ++b)
    for (int a = 0; a < NP; ++a) {
      const double ph = tb.L[qi][a] * tb.L[qj][b], px = tb.D[qi][a] * tb.L[qj][b], py = tb.L[qi][a] * tb.D[qj][b];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = ue[v * NN + a + NP * b], r = re[v * NN + a + NP * b];
        W[v] += ph * x;
        G[v][0] += px * x * sx;
        G[v][1] += py * x * sy;
        rx[v] += px * r;
        ry[v] += py * r;
      }
    }
  const double w = tb.W[qi] * tb.W[qj];
  double Fb[4][2];
#pragma unroll
  for (int v = 0; v < 4; ++v) { Fb[v][0] = w * 0.5 * hy * rx[v]; Fb[v][1] = w * 0.5 * hx * ry[v]; }
  double xb[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) xb[i] = 0.0;
  using D4 = Dual<4>;
  const int nchunk = g.viscous ? 3 : 1;
  for (int ch = 0; ch < nchunk; ++ch) {
    D4 Wd[4], Gd[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wd[v] = D4(W[v]);
      const int idx = v - 4 * ch;
      if (idx >= 0 && idx < 4) Wd[v].d[idx] = 1.0;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        Gd[v][d] = D4(G[v][d]);
        const int jdx = 4 + 2 * v + d - 4 * ch;
        if (jdx >= 0 && jdx < 4) Gd[v][d].d[jdx] = 1.0;
      }
    }
    D4 Fc[4][2], F[4][2];
    conv_flux(Wd, g, Fc);
#pragma unroll
    for (int v = 0; v < 4; ++v) { F[v][0] = -Fc[v][0]; F[v][1] = -Fc[v][1]; }
    if (g.viscous) {
      D4 Fv[4][2];
      visc_flux(Wd, Gd, g, Fv);
#pragma unroll
      for (int v = 0; v < 4; ++v) { F[v][0] = F[v][0] + Fv[v][0]; F[v][1] = F[v][1] + Fv[v][1]; }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int col = 4 * ch + k;
      if (col >= 12) break;
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc += Fb[v][0] * F[v][0].d[k] + Fb[v][1] * F[v][1].d[k];
      xb[col] += acc;
    }
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) out[i] = xb[i];
}

// 4. Ubar[e][v][n] = sum over points of phi_n Wbar_v + (2/hx) dphi_n/dxi Gbar_v,x + (2/hy) dphi_n/deta Gbar_v,y
template <int K>
__global__ void __launch_bounds__(256) vjp_contract_kernel(DeviceMesh m, const double* __restrict__ PV,
                                                           const double* __restrict__ PF, double* __restrict__ Ub) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP, NQV = NQ * NQ;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * NN) return;
  const int n = t % NN, e = t / NN;
  const int a = n % NP, b = n / NP;
  const BasisTable& tb = *m.tab;
  const double sx = 2.0 / m.hx[e], sy = 2.0 / m.hy[e];
  double r[4] = {0, 0, 0, 0};
  if (!m.imp[e]) {
    const double* pv = PV + (size_t)e * NQV * 12;
    for (int qj = 0; qj < NQ; ++qj)
      for (int qi = 0; qi < NQ; ++qi) {
        const double* p = pv + (qi + NQ * qj) * 12;
        const double ph = tb.L[qi][a] * tb.L[qj][b];
        const double px = tb.D[qi][a] * tb.L[qj][b] * sx, py = tb.L[qi][a] * tb.D[qj][b] * sy;
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] += ph * p[v] + px * p[4 + 2 * v] + py * p[5 + 2 * v];
      }
  }
  const double* pf = PF + (size_t)e * 4 * NQ * 12;
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
      const double* p = pf + (f * NQ + q) * 12;
#pragma unroll
      for (int v = 0; v < 4; ++v) r[v] += ph * p[v] + pxi * sx * p[4 + 2 * v] + peta * sy * p[5 + 2 * v];
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Ub[(size_t)e * 4 * NN + v * NN + n] = r[v];
}

// Qbar[e][c][n] = sum over face points of phi_n PQ[e][f][q][c] (HDG-MX implicit elements)
template <int K>
__global__ void vjp_qcontract_kernel(DeviceMesh m, const double* __restrict__ PQ, double* __restrict__ Qb) {
  constexpr int NP = K + 1, NQ = (3 * K + 2) / 2, NN = NP * NP;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.E * NN) return;
  const int e = t / NN, n = t % NN, a = n % NP, b = n / NP;
  if (!m.imp[e]) return;
  const BasisTable& tb = *m.tab;
  double r[5] = {0, 0, 0, 0, 0};
  for (int f = 0; f < 4; ++f) {
    const int s = f & 1;
    for (int q = 0; q < NQ; ++q) {
      const double ph = (f < 2) ? tb.LE[s][a] * tb.L[q][b] : tb.L[q][a] * tb.LE[s][b];
      const double* pq = PQ + (((size_t)e * 4 + f) * NQ + q) * 5;
#pragma unroll
      for (int c = 0; c < 5; ++c) r[c] += ph * pq[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) Qb[(size_t)e * 5 * NN + c * NN + n] = r[c];
}

#define VJP_DISPATCH(KV, ...)                                   \
  switch (KV) {                                                 \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;       \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;       \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;       \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;       \
    default: return hipErrorInvalidValue;                       \
  }

hipError_t vjp_alloc(imex_ctx* c) {
  Workspace& w = c->ws;
  if (w.vjp_tu) return hipSuccess;
  const size_t E = c->E, NQ = c->NQ, NN = c->NN;
  const size_t nf = E * 4 * NQ * 12, nv = E * NQ * NQ * 12, es = E * 4 * NN;
  hipError_t e = hipMalloc(&w.vjp_tu, 8 * nf);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_tr, 8 * nf);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_pf, 8 * nf);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_pv, 8 * nv);
  for (int i = 0; i < 10 && e == hipSuccess; ++i) e = hipMalloc(&w.vjp_y[i], 8 * es);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_tq, 8 * E * 4 * NQ * 5);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_pq, 8 * E * 4 * NQ * 5);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_qb, 8 * E * 5 * NN);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_q, 8 * E * 5 * NN);
  if (e == hipSuccess) e = hipMalloc(&w.vjp_hb, 8 * std::max<size_t>((size_t)c->n_im * 16 * c->NP, 1));
  if (e == hipSuccess) e = hipMemsetAsync(w.vjp_q, 0, 8 * E * 5 * NN, c->stream);
  if (e == hipSuccess) w.bytes += 8 * (3 * nf + nv + 10 * es + 2 * E * 4 * NQ * 5 + 2 * E * 5 * NN);
  return e;
}

// Ubar = (dR^DG/dU)^T Rbar; with HDG-MX coupling (Uhat given) the implicit side's mixed
// variables are lifted from (U, Uhat) and their adjoint is taken back through the lifting:
// Ubar (implicit rows) and Uhatbar (added) receive it.
hipError_t launch_dg_vjp(imex_ctx* c, const double* U, const double* Rb, double* Ub, const double* Uhat,
                         double* Uhatbar) {
  Workspace& w = c->ws;
  const int nfp = c->E * 4 * c->NQ, nvp = c->E * c->NQ * c->NQ, nn = c->E * c->NN;
  const int lf = c->opt.dg_flux == IMEX_FLUX_LAX_FRIEDRICHS;
  const bool mx = Uhat && c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous && c->n_im > 0;
  if (mx) {
    hipError_t e = launch_lift_mixed(c, U, Uhat, w.vjp_q);
    if (e != hipSuccess) return e;
  }
  double* TQ = mx ? w.vjp_tq : nullptr;
  double* PQ = mx ? w.vjp_pq : nullptr;
  VJP_DISPATCH(c->K, {
    hipLaunchKernelGGL(vjp_trace_kernel<KK>, dim3((nfp + 255) / 256), dim3(256), 0, c->stream, c->dmesh(), U, Rb,
                       w.vjp_tu, w.vjp_tr, mx ? w.vjp_q : nullptr, TQ);
    hipLaunchKernelGGL(vjp_face_kernel<KK>, dim3((nfp + 127) / 128), dim3(128), 0, c->stream, c->dmesh(), c->gas, lf,
                       c->opt.alpha_dg, w.vjp_tu, w.vjp_tr, w.vjp_pf, TQ, PQ);
    hipLaunchKernelGGL(vjp_volume_kernel<KK>, dim3((nvp + 127) / 128), dim3(128), 0, c->stream, c->dmesh(), c->gas,
                       U, Rb, w.vjp_pv);
    hipLaunchKernelGGL(vjp_contract_kernel<KK>, dim3((nn + 255) / 256), dim3(256), 0, c->stream, c->dmesh(),
                       w.vjp_pv, w.vjp_pf, Ub);
    if (mx) {
      hipLaunchKernelGGL(vjp_qcontract_kernel<KK>, dim3((nn + 255) / 256), dim3(256), 0, c->stream, c->dmesh(), PQ,
                         w.vjp_qb);
    }
  });
  if (mx) return launch_lift_vjp(c, U, Uhat, w.vjp_qb, Ub, w.vjp_hb, Uhatbar);
  return hipGetLastError();
}

}  // namespace imex
