// Explicit DG-IP residual on hexahedra (the three-dimensional form of
// eq. bilinear_form_interior_sdg with five conservative variables): the explicit part of
// the 3D channel.  The paper's forms are two-dimensional; the 3D form adds the third
// direction term by term (convective and viscous fluxes of Sec. 2 with lambda = -2 mu / 3,
// Vijayasundaram or Lax-Friedrichs faces, interior-penalty consistency, adjoint and penalty
// terms, far-field faces as in App. B.1.1).
//
// Kernels (one workgroup of 128 threads per element):
//  * dg3d_trace_kernel: the element's traces on its six faces.  The nodal values are
//    first contracted with the end values (and end derivatives) of the 1D basis along the
//    face normal, then interpolated to the face's Gauss points; each face point stores
//    U and, with viscosity, F^nu(U, grad U) . n (at U_inf on far-field faces).
//  * dg3d_residual_kernel: volume term by sum factorisation (three 1D passes to the Gauss
//    points for the state and its gradient, point fluxes, three transposed passes back to
//    the nodes, all through LDS); face terms at each face point from the own and the
//    neighbour's trace records (numerical flux, consistency, penalty, and the adjoint term
//    tested against grad V), lifted to the nodes by a 2D contraction per face and the end
//    values along the normal.
// Layout: U[e][v][n], n = a + N b + N^2 c (x fastest), element e = i + nx (j + ny l);
// records rec[e][f][p][RS], faces f = x-, x+, y-, y+, z-, z+, face point p = i1 + Q i2
// over the two tangential axes in increasing axis order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "device_common.h"
#include "imexhdg.h"

namespace imex {
void basis_table_1d(int K, BasisTable& T);
void gauss_legendre_rule(int n, double* x, double* w);

constexpr int NT3 = 128;

struct Gas3D {
  double gamma, R, mu, Pr, cv, kappa, lam;
  int viscous;
  double uinf[5];
};

struct Mesh3D {
  int nx, ny, nz, E;
  const int* nbr;        // [E][6] neighbour element or -1
  const int* bc;         // [E][6] boundary type where nbr < 0
  const double* h;       // [E][3] element sizes
  const double* lchar;   // [E] |T| / |dT|
};

template <int K> struct S3 {
  static constexpr int N = K + 1, Q = (3 * K + 2) / 2, NN = N * N * N, QQ = Q * Q, QQQ = Q * Q * Q, NF2 = N * N;
};

// ---------------------------------------------------------------------------
// physics
// ---------------------------------------------------------------------------
__device__ inline void conv3(const double U[5], const Gas3D& g, double F[5][3]) {
  const double rho = U[0], ir = 1.0 / rho;
  const double u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
  const double p = (g.gamma - 1.0) * (U[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F[0][d] = U[1 + d];
#pragma unroll
    for (int m = 0; m < 3; ++m) F[1 + m][d] = U[1 + m] * u[d] + (m == d ? p : 0.0);
    F[4][d] = (U[4] + p) * u[d];
  }
}

// F^nu at state W with the conservative gradient replaced by G (= K(W) G)
__device__ inline void visc3(const double W[5], const double G[5][3], const Gas3D& g, double F[5][3]) {
  const double ir = 1.0 / W[0];
  const double u[3] = {W[1] * ir, W[2] * ir, W[3] * ir};
  const double E = W[4] * ir;
  double gu[3][3], gt[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int m = 0; m < 3; ++m) gu[m][d] = (G[1 + m][d] - u[m] * G[0][d]) * ir;
    const double gE = (G[4][d] - E * G[0][d]) * ir;
    gt[d] = (gE - u[0] * gu[0][d] - u[1] * gu[1][d] - u[2] * gu[2][d]) / g.cv;
  }
  const double div = gu[0][0] + gu[1][1] + gu[2][2];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F[0][d] = 0.0;
    double e = g.kappa * gt[d];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double t = g.mu * (gu[m][d] + gu[d][m]) + (m == d ? g.lam * div : 0.0);
      F[1 + m][d] = t;
      e += t * u[m];
    }
    F[4][d] = e;
  }
}

// K(W) (J (x) n) . n
__device__ inline void visc3_jump_n(const double W[5], const double J[5], const double n[3], const Gas3D& g,
                                    double out[5], double Fj[5][3]) {
  double G[5][3];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int d = 0; d < 3; ++d) G[v][d] = J[v] * n[d];
  visc3(W, G, g, Fj);
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = Fj[v][0] * n[0] + Fj[v][1] * n[1] + Fj[v][2] * n[2];
}

// out += A^+-(Wbar) X (sign +1: A^+, -1: A^-) by the characteristic decomposition of X at
// Wbar: acoustic amplitudes (dp -+ rho c du_n) / (2 c^2), entropy drho - dp / c^2 and the
// tangential velocity, each scaled by the positive or negative part of its eigenvalue.
__device__ inline void apply_split3(const double Wb[5], const double X[5], const double n[3], double sign,
                                    const Gas3D& g, double out[5]) {
  const double rho = Wb[0], ir = 1.0 / rho;
  const double u[3] = {Wb[1] * ir, Wb[2] * ir, Wb[3] * ir};
  const double q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double p = (g.gamma - 1.0) * (Wb[4] - 0.5 * rho * q2);
  const double c2 = g.gamma * p * ir, c = sqrt(c2);
  const double H = (Wb[4] + p) * ir;
  const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  double du[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) du[m] = (X[1 + m] - u[m] * X[0]) * ir;
  const double dp = (g.gamma - 1.0) * (X[4] - (u[0] * X[1] + u[1] * X[2] + u[2] * X[3]) + 0.5 * q2 * X[0]);
  const double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const double am = (dp - rho * c * dun) / (2.0 * c2), ap = (dp + rho * c * dun) / (2.0 * c2);
  const double a0 = X[0] - dp / c2;
  double dut[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) dut[m] = du[m] - dun * n[m];
  auto part = [&](double l) { return sign > 0.0 ? (l > 0.0 ? l : 0.0) : (l < 0.0 ? l : 0.0); };
  const double lm = part(un - c) * am, l0 = part(un), lp = part(un + c) * ap;
  out[0] += lm + l0 * a0 + lp;
#pragma unroll
  for (int m = 0; m < 3; ++m) out[1 + m] += lm * (u[m] - c * n[m]) + l0 * (a0 * u[m] + rho * dut[m]) + lp * (u[m] + c * n[m]);
  out[4] += lm * (H - c * un) + l0 * (a0 * 0.5 * q2 + rho * (u[0] * dut[0] + u[1] * dut[1] + u[2] * dut[2])) +
            lp * (H + c * un);
}

__device__ inline double wave_speed3(const double W[5], const double n[3], const Gas3D& g) {
  const double ir = 1.0 / W[0];
  const double u[3] = {W[1] * ir, W[2] * ir, W[3] * ir};
  const double p = (g.gamma - 1.0) * (W[4] - 0.5 * W[0] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  return fabs(un) + sqrt(g.gamma * p * ir);
}

// ---------------------------------------------------------------------------
// trace kernel
// ---------------------------------------------------------------------------
template <int K>
__global__ void __launch_bounds__(NT3) dg3d_trace_kernel(Mesh3D m, Gas3D g, BasisTable tb, const double* __restrict__ U,
                                                        double* __restrict__ rec, int RS) {
  using S = S3<K>;
  constexpr int N = S::N, Q = S::Q, NN = S::NN, QQ = S::QQ, NF2 = S::NF2;
  __shared__ double su[5][NN];
  __shared__ double ec[6][2][5][NF2];      // end contractions: value / normal derivative
  const int e = blockIdx.x, t = threadIdx.x;
  for (int i = t; i < 5 * NN; i += NT3) su[i / NN][i % NN] = U[(size_t)e * 5 * NN + i];
  __syncthreads();
  for (int i = t; i < 6 * 2 * 5 * NF2; i += NT3) {
    const int f = i / (10 * NF2), r = i % (10 * NF2), kind = r / (5 * NF2), v = (r / NF2) % 5, tt = r % NF2;
    const int d = f >> 1, s = f & 1;
    const int j1 = tt % N, j2 = tt / N;     // tangential node indices (first, second tangential axis)
    // node strides of the normal and the two tangential axes
    const int sd = d == 0 ? 1 : (d == 1 ? N : N * N);
    const int s1 = d == 0 ? N : 1, s2 = d == 2 ? N : N * N;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const double wgt = kind == 0 ? tb.LE[s][a] : tb.DE[s][a];
      acc += wgt * su[v][a * sd + j1 * s1 + j2 * s2];
    }
    ec[f][kind][v][tt] = acc;
  }
  __syncthreads();
  const double* h = m.h + 3 * (size_t)e;
  for (int i = t; i < 6 * QQ; i += NT3) {
    const int f = i / QQ, pnt = i % QQ, d = f >> 1;
    const int i1 = pnt % Q, i2 = pnt / Q;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    double Uf[5], G[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double val = 0.0, g1 = 0.0, g2 = 0.0, gn = 0.0;
#pragma unroll
      for (int j2 = 0; j2 < N; ++j2)
#pragma unroll
        for (int j1 = 0; j1 < N; ++j1) {
          const double x0 = ec[f][0][v][j1 + N * j2], x1 = ec[f][1][v][j1 + N * j2];
          const double L1 = tb.L[i1][j1], L2 = tb.L[i2][j2];
          val += L1 * L2 * x0;
          g1 += tb.D[i1][j1] * L2 * x0;
          g2 += L1 * tb.D[i2][j2] * x0;
          gn += L1 * L2 * x1;
        }
      Uf[v] = val;
      const double vn = gn * 2.0 / h[d], v1 = g1 * 2.0 / h[t1], v2 = g2 * 2.0 / h[t2];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) G[v][ax] = ax == d ? vn : (ax == t1 ? v1 : v2);
    }
    double* r = rec + (((size_t)e * 6 + f) * QQ + pnt) * RS;
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] = Uf[v];
    if (RS > 5) {
      const bool far = m.nbr[6 * (size_t)e + f] < 0 && m.bc[6 * (size_t)e + f] == IMEX_BC_FARFIELD;
      const double sg = (f & 1) ? 1.0 : -1.0;
      const double n[3] = {d == 0 ? sg : 0.0, d == 1 ? sg : 0.0, d == 2 ? sg : 0.0};
      double F[5][3], Ws[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Ws[v] = far ? g.uinf[v] : Uf[v];
      visc3(Ws, G, g, F);
#pragma unroll
      for (int v = 0; v < 5; ++v) r[5 + v] = F[v][0] * n[0] + F[v][1] * n[1] + F[v][2] * n[2];
    }
  }
}

// ---------------------------------------------------------------------------
// residual kernel
// ---------------------------------------------------------------------------
template <int K, bool VISC>
__global__ void __launch_bounds__(NT3) dg3d_residual_kernel(Mesh3D m, Gas3D g, BasisTable tb, int flux, double alpha,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ rec, int RS,
                                                           double* __restrict__ R) {
  using S = S3<K>;
  constexpr int N = S::N, Q = S::Q, NN = S::NN, QQ = S::QQ, QQQ = S::QQQ, NF2 = S::NF2;
  constexpr int NX = 5 * 2 * Q * N * N, NY = 5 * 3 * Q * Q * N, NQ4 = 5 * 4 * QQQ;
  constexpr int NFB = 6 * 5 * QQ * 4;                    // face buffers: s and g per face point
  constexpr int BIG = NQ4 > NFB ? NQ4 : NFB;
  constexpr int NHB = 6 * 5 * 2 * NF2;                   // per-face 2D contractions (after the volume passes)
  constexpr int NTY = NY > NHB ? NY : NHB;
  __shared__ double su[5 * NN], rv[5 * NN];
  __shared__ double tx[NX], ty[NTY], big[BIG];
  double* hb = ty;                                       // ty is free once the transposed y pass has run
  const int e = blockIdx.x, t = threadIdx.x;
  const double* h = m.h + 3 * (size_t)e;
  const double hx = h[0], hy = h[1], hz = h[2];
  const double jac = hx * hy * hz / 8.0;
  for (int i = t; i < 5 * NN; i += NT3) su[i] = U[(size_t)e * 5 * NN + i];
  __syncthreads();
  // volume: pass along x (value, derivative)
  for (int i = t; i < NX; i += NT3) {
    const int v = i / (2 * Q * N * N), r = i % (2 * Q * N * N), kind = r / (Q * N * N), rr = r % (Q * N * N);
    const int qx = rr % Q, b = (rr / Q) % N, c = rr / (Q * N);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) acc += (kind == 0 ? tb.L[qx][a] : tb.D[qx][a]) * su[v * NN + a + N * b + N * N * c];
    tx[i] = acc;                                          // tx[v][kind][c][b][qx]
  }
  __syncthreads();
  // pass along y: (x-value, y) -> value, d/dy; (x-deriv, y) -> d/dx
  for (int i = t; i < NY; i += NT3) {
    const int v = i / (3 * Q * Q * N), r = i % (3 * Q * Q * N), kind = r / (Q * Q * N), rr = r % (Q * Q * N);
    const int qx = rr % Q, qy = (rr / Q) % Q, c = rr / (Q * Q);
    const double* src = tx + (size_t)v * 2 * Q * N * N + (kind == 1 ? Q * N * N : 0);
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) acc += (kind == 2 ? tb.D[qy][b] : tb.L[qy][b]) * src[qx + Q * b + Q * N * c];
    ty[i] = acc;                                          // ty[v][kind][c][qy][qx]: 0 value, 1 d/dx, 2 d/dy
  }
  __syncthreads();
  // pass along z: value, d/dx, d/dy, d/dz at the volume points
  for (int i = t; i < NQ4; i += NT3) {
    const int v = i / (4 * QQQ), r = i % (4 * QQQ), kind = r / QQQ, q = r % QQQ;
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / QQ;
    const int sk = kind == 3 ? 0 : kind;
    const double* src = ty + (size_t)v * 3 * Q * Q * N + sk * Q * Q * N;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c) acc += (kind == 3 ? tb.D[qz][c] : tb.L[qz][c]) * src[qx + Q * qy + QQ * c];
    big[i] = acc;                                         // big[v][kind][q]
  }
  __syncthreads();
  // point fluxes, scaled by the quadrature weight, |J| and d xi_d / d x_d
  const double sc[3] = {2.0 / hx, 2.0 / hy, 2.0 / hz};
  for (int q = t; q < QQQ; q += NT3) {
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / QQ;
    const double w = tb.W[qx] * tb.W[qy] * tb.W[qz] * jac;
    double Uq[5], G[5][3], F[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Uq[v] = big[(v * 4 + 0) * QQQ + q];
#pragma unroll
      for (int d = 0; d < 3; ++d) G[v][d] = big[(v * 4 + 1 + d) * QQQ + q] * sc[d];
    }
    conv3(Uq, g, F);
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) F[v][d] = -F[v][d];
    if (VISC) {
      double Fv[5][3];
      visc3(Uq, G, g, Fv);
#pragma unroll
      for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) F[v][d] += Fv[v][d];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) big[(v * 4 + d) * QQQ + q] = F[v][d] * w * sc[d];
  }
  __syncthreads();
  // transposed pass along z: (Gx, Gy) with L, Gz with D -> ty[v][3][c][qy][qx]
  for (int i = t; i < NY; i += NT3) {
    const int v = i / (3 * Q * Q * N), r = i % (3 * Q * Q * N), kind = r / (Q * Q * N), rr = r % (Q * Q * N);
    const int qx = rr % Q, qy = (rr / Q) % Q, c = rr / (Q * Q);
    const double* src = big + (size_t)(v * 4 + kind) * QQQ;
    double acc = 0.0;
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) acc += (kind == 2 ? tb.D[qz][c] : tb.L[qz][c]) * src[qx + Q * qy + QQ * qz];
    ty[i] = acc;
  }
  __syncthreads();
  // transposed pass along y: Bx = sum L Ax, Byz = sum D Ay + L Az -> tx[v][2][c][b][qx]
  for (int i = t; i < NX; i += NT3) {
    const int v = i / (2 * Q * N * N), r = i % (2 * Q * N * N), kind = r / (Q * N * N), rr = r % (Q * N * N);
    const int qx = rr % Q, b = (rr / Q) % N, c = rr / (Q * N);
    const double* A = ty + (size_t)v * 3 * Q * Q * N;
    double acc = 0.0;
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      const int o = qx + Q * qy + Q * Q * c;
      if (kind == 0) acc += tb.L[qy][b] * A[o];
      else acc += tb.D[qy][b] * A[Q * Q * N + o] + tb.L[qy][b] * A[2 * Q * Q * N + o];
    }
    tx[i] = acc;
  }
  __syncthreads();
  // transposed pass along x: R = sum D Bx + L Byz
  for (int i = t; i < 5 * NN; i += NT3) {
    const int v = i / NN, n = i % NN, a = n % N, b = (n / N) % N, c = n / (N * N);
    const double* B = tx + (size_t)v * 2 * Q * N * N;
    double acc = 0.0;
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) {
      const int o = qx + Q * b + Q * N * c;
      acc += tb.D[qx][a] * B[o] + tb.L[qx][a] * B[Q * N * N + o];
    }
    rv[i] = acc;
  }
  __syncthreads();
  // face points: s tested against V, g against grad V (weights and metric folded in)
  const double kk = (K + 1) * (K + 1);
  const double lown = m.lchar[e];
  for (int i = t; i < 6 * QQ; i += NT3) {
    const int f = i / QQ, pnt = i % QQ, d = f >> 1;
    const int i1 = pnt % Q, i2 = pnt / Q;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    double n[3] = {0.0, 0.0, 0.0};
    n[d] = (f & 1) ? 1.0 : -1.0;
    const int nb = m.nbr[6 * (size_t)e + f];
    const bool far = nb < 0 && m.bc[6 * (size_t)e + f] == IMEX_BC_FARFIELD;
    const double* ro = rec + (((size_t)e * 6 + f) * QQ + pnt) * RS;
    double Uo[5], Un[5], s[5], gg[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v) Uo[v] = ro[v];
    const double* rn = nullptr;
    if (nb >= 0) {
      rn = rec + (((size_t)nb * 6 + (f ^ 1)) * QQ + pnt) * RS;
#pragma unroll
      for (int v = 0; v < 5; ++v) Un[v] = rn[v];
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) Un[v] = g.uinf[v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      s[v] = 0.0;
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) gg[v][dd] = 0.0;
    }
    if (far) {
      apply_split3(Uo, Uo, n, 1.0, g, s);
      apply_split3(Uo, Un, n, -1.0, g, s);
    } else if (flux == IMEX_FLUX_LAX_FRIEDRICHS) {
      double Fa[5][3], Fb[5][3];
      conv3(Uo, g, Fa);
      conv3(Un, g, Fb);
      const double la = wave_speed3(Uo, n, g), lb = wave_speed3(Un, n, g), lam = la > lb ? la : lb;
#pragma unroll
      for (int v = 0; v < 5; ++v)
        s[v] = 0.5 * (Fa[v][d] + Fb[v][d]) * n[d] + 0.5 * lam * (Uo[v] - Un[v]);
    } else {
      double Wb[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Wb[v] = 0.5 * (Uo[v] + Un[v]);
      apply_split3(Wb, Uo, n, 1.0, g, s);
      apply_split3(Wb, Un, n, -1.0, g, s);
    }
    if (VISC) {
      double J[5], pa[5], pb[5], Fa[5][3], Fb[5][3];
#pragma unroll
      for (int v = 0; v < 5; ++v) J[v] = Uo[v] - Un[v];
      if (far) {
        const double tau = alpha * kk / lown;
        visc3_jump_n(g.uinf, J, n, g, pa, Fa);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          s[v] += -ro[5 + v] + tau * pa[v];
#pragma unroll
          for (int dd = 0; dd < 3; ++dd) gg[v][dd] = -Fa[v][dd];
        }
      } else {
        const double lmin = (nb >= 0 && m.lchar[nb] < lown) ? m.lchar[nb] : lown;
        const double tau = alpha * kk / lmin;
        visc3_jump_n(Uo, J, n, g, pa, Fa);
        visc3_jump_n(Un, J, n, g, pb, Fb);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          // the neighbour's record holds F^nu . (its own outward normal) = -F^nu . n
          s[v] += -0.5 * (ro[5 + v] - rn[5 + v]) + tau * 0.5 * (pa[v] + pb[v]);
#pragma unroll
          for (int dd = 0; dd < 3; ++dd) gg[v][dd] = -0.5 * Fa[v][dd];
        }
      }
    }
    const double wf = tb.W[i1] * tb.W[i2] * (h[t1] * h[t2] / 4.0);
    double* fb = big + (size_t)(f * 5) * QQ * 4;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      fb[(v * 4 + 0) * QQ + pnt] = s[v] * wf;
      fb[(v * 4 + 1) * QQ + pnt] = gg[v][t1] * wf * 2.0 / h[t1];
      fb[(v * 4 + 2) * QQ + pnt] = gg[v][t2] * wf * 2.0 / h[t2];
      fb[(v * 4 + 3) * QQ + pnt] = gg[v][d] * wf * 2.0 / h[d];
    }
  }
  __syncthreads();
  // per face: Hval[j1][j2] = sum L L s + D L g_t1 + L D g_t2, Hn[j1][j2] = sum L L g_n
  for (int i = t; i < 6 * 5 * NF2; i += NT3) {
    const int f = i / (5 * NF2), v = (i / NF2) % 5, tt = i % NF2;
    const int j1 = tt % N, j2 = tt / N;
    const double* fb = big + ((size_t)(f * 5 + v) * 4) * QQ;
    double hv = 0.0, hn = 0.0;
#pragma unroll
    for (int i2 = 0; i2 < Q; ++i2)
#pragma unroll
      for (int i1 = 0; i1 < Q; ++i1) {
        const int p = i1 + Q * i2;
        const double L1 = tb.L[i1][j1], L2 = tb.L[i2][j2];
        hv += L1 * L2 * fb[p] + tb.D[i1][j1] * L2 * fb[QQ + p] + L1 * tb.D[i2][j2] * fb[2 * QQ + p];
        hn += L1 * L2 * fb[3 * QQ + p];
      }
    hb[((f * 5 + v) * 2 + 0) * NF2 + tt] = hv;
    hb[((f * 5 + v) * 2 + 1) * NF2 + tt] = hn;
  }
  __syncthreads();
  for (int i = t; i < 5 * NN; i += NT3) {
    const int v = i / NN, n = i % NN;
    const int idx[3] = {n % N, (n / N) % N, n / (N * N)};
    double acc = rv[i];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      const int j1 = idx[d == 0 ? 1 : 0], j2 = idx[d == 2 ? 1 : 2];
      const int o = ((f * 5 + v) * 2) * NF2 + j1 + N * j2;
      acc += tb.LE[s][idx[d]] * hb[o] + tb.DE[s][idx[d]] * hb[o + NF2];
    }
    R[(size_t)e * 5 * NN + i] = acc;
  }
}
}  // namespace imex

using namespace imex;

struct imex3d_ctx {
  int nx = 0, ny = 0, nz = 0, E = 0, K = 0, flux = 0;
  double alpha = 1.0;
  Gas3D gas{};
  BasisTable tab{};
  hipStream_t stream = nullptr;
  int* d_nbr = nullptr;
  int* d_bc = nullptr;
  double* d_h = nullptr;
  double* d_lchar = nullptr;
  double* d_rec = nullptr;
  std::vector<double> x, y, z;
  std::string err;
};

static imex_status fail3(imex3d_ctx* c, imex_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP3(c, expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail3(c, IMEX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" {

imex_status imex3d_create(const imex3d_mesh_desc* mesh, const imex_physics* phys, int dg_flux, double alpha_dg,
                          const double u_inf[5], void* stream, imex3d_ctx** out) {
  if (!mesh || !phys || !u_inf || !out) return fail3(nullptr, IMEX_EINVAL, "null argument");
  *out = nullptr;
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 || !mesh->xgrid || !mesh->ygrid || !mesh->zgrid)
    return IMEX_EINVAL;
  if (mesh->degree < 1 || mesh->degree > 3) return IMEX_EINVAL;
  if (dg_flux != IMEX_FLUX_VIJAYASUNDARAM && dg_flux != IMEX_FLUX_LAX_FRIEDRICHS) return IMEX_EINVAL;
  for (int s = 0; s < 6; ++s) {
    if (mesh->bc[s] != IMEX_BC_PERIODIC && mesh->bc[s] != IMEX_BC_FARFIELD) return IMEX_EINVAL;
    if ((mesh->bc[s] == IMEX_BC_PERIODIC) != (mesh->bc[s ^ 1] == IMEX_BC_PERIODIC)) return IMEX_EINVAL;
  }
  const int dims[3] = {mesh->nx, mesh->ny, mesh->nz};
  const double* grids[3] = {mesh->xgrid, mesh->ygrid, mesh->zgrid};
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < dims[d]; ++i)
      if (!(grids[d][i + 1] > grids[d][i])) return IMEX_EINVAL;
  if (!(phys->gamma > 1.0) || !(phys->R > 0.0) || !(phys->mu >= 0.0) || !(phys->Pr > 0.0)) return IMEX_EINVAL;
  auto* c = new imex3d_ctx();
  c->nx = mesh->nx;
  c->ny = mesh->ny;
  c->nz = mesh->nz;
  c->E = c->nx * c->ny * c->nz;
  c->K = mesh->degree;
  c->flux = dg_flux;
  c->alpha = alpha_dg;
  c->stream = static_cast<hipStream_t>(stream);
  c->x.assign(mesh->xgrid, mesh->xgrid + c->nx + 1);
  c->y.assign(mesh->ygrid, mesh->ygrid + c->ny + 1);
  c->z.assign(mesh->zgrid, mesh->zgrid + c->nz + 1);
  Gas3D& g = c->gas;
  g.gamma = phys->gamma;
  g.R = phys->R;
  g.mu = phys->viscous ? phys->mu : 0.0;
  g.Pr = phys->Pr;
  g.cv = phys->R / (phys->gamma - 1.0);
  g.kappa = phys->gamma * g.cv * g.mu / phys->Pr;
  g.lam = -2.0 * g.mu / 3.0;
  g.viscous = phys->viscous ? 1 : 0;
  for (int v = 0; v < 5; ++v) g.uinf[v] = u_inf[v];
  basis_table_1d(c->K, c->tab);
  const int E = c->E;
  std::vector<int> nbr(6 * (size_t)E), bc(6 * (size_t)E);
  std::vector<double> hh(3 * (size_t)E), lch(E);
  for (int e = 0; e < E; ++e) {
    const int ijl[3] = {e % c->nx, (e / c->nx) % c->ny, e / (c->nx * c->ny)};
    double hd[3];
    for (int d = 0; d < 3; ++d) hd[d] = grids[d][ijl[d] + 1] - grids[d][ijl[d]];
    for (int d = 0; d < 3; ++d) hh[3 * (size_t)e + d] = hd[d];
    lch[e] = hd[0] * hd[1] * hd[2] / (2.0 * (hd[0] * hd[1] + hd[1] * hd[2] + hd[2] * hd[0]));
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      int idx[3] = {ijl[0], ijl[1], ijl[2]};
      idx[d] += s ? 1 : -1;
      const bool inside = idx[d] >= 0 && idx[d] < dims[d];
      const bool per = mesh->bc[f] == IMEX_BC_PERIODIC;
      idx[d] = (idx[d] % dims[d] + dims[d]) % dims[d];
      if (inside || per) {
        nbr[6 * (size_t)e + f] = idx[0] + c->nx * (idx[1] + c->ny * idx[2]);
        bc[6 * (size_t)e + f] = -1;
      } else {
        nbr[6 * (size_t)e + f] = -1;
        bc[6 * (size_t)e + f] = mesh->bc[f];
      }
    }
  }
  const int N = c->K + 1, Q = (3 * c->K + 2) / 2;
  const size_t recsz = (size_t)E * 6 * Q * Q * 10;
  hipError_t he = hipMalloc(&c->d_nbr, sizeof(int) * nbr.size());
  if (he == hipSuccess) he = hipMalloc(&c->d_bc, sizeof(int) * bc.size());
  if (he == hipSuccess) he = hipMalloc(&c->d_h, sizeof(double) * hh.size());
  if (he == hipSuccess) he = hipMalloc(&c->d_lchar, sizeof(double) * lch.size());
  if (he == hipSuccess) he = hipMalloc(&c->d_rec, sizeof(double) * recsz);
  if (he != hipSuccess) {
    imex3d_destroy(c);
    return IMEX_ENOMEM;
  }
  (void)N;
  he = hipMemcpy(c->d_nbr, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(c->d_bc, bc.data(), sizeof(int) * bc.size(), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(c->d_h, hh.data(), sizeof(double) * hh.size(), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(c->d_lchar, lch.data(), sizeof(double) * lch.size(), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    imex3d_destroy(c);
    return IMEX_EDEVICE;
  }
  *out = c;
  return IMEX_OK;
}

imex_status imex3d_query_sizes(const imex3d_ctx* c, long long out[4]) {
  if (!c || !out) return IMEX_EINVAL;
  const int N = c->K + 1, Q = (3 * c->K + 2) / 2;
  out[0] = c->E;
  out[1] = (long long)N * N * N;
  out[2] = Q;
  out[3] = (long long)c->E * 6 * Q * Q * 10 * 8;
  return IMEX_OK;
}

imex_status imex3d_node_coords(const imex3d_ctx* c, double* x, double* y, double* z) {
  if (!c || !x || !y || !z) return IMEX_EINVAL;
  const int N = c->K + 1;
  double nodes[MAXNP], nw[MAXNP];
  gauss_legendre_rule(N, nodes, nw);
  const int NN = N * N * N;
  for (int e = 0; e < c->E; ++e) {
    const int i = e % c->nx, j = (e / c->nx) % c->ny, l = e / (c->nx * c->ny);
    for (int n = 0; n < NN; ++n) {
      const int a = n % N, b = (n / N) % N, cc = n / (N * N);
      x[(size_t)e * NN + n] = c->x[i] + 0.5 * (nodes[a] + 1.0) * (c->x[i + 1] - c->x[i]);
      y[(size_t)e * NN + n] = c->y[j] + 0.5 * (nodes[b] + 1.0) * (c->y[j + 1] - c->y[j]);
      z[(size_t)e * NN + n] = c->z[l] + 0.5 * (nodes[cc] + 1.0) * (c->z[l + 1] - c->z[l]);
    }
  }
  return IMEX_OK;
}

imex_status imex3d_residual(imex3d_ctx* c, const double* U, double* R) {
  if (!c || !U || !R) return fail3(c, IMEX_EINVAL, "null argument");
  const Mesh3D m{c->nx, c->ny, c->nz, c->E, c->d_nbr, c->d_bc, c->d_h, c->d_lchar};
  const int RS = c->gas.viscous ? 10 : 5;
  const bool visc = c->gas.viscous != 0;
#define DG3_LAUNCH(KK)                                                                                         \
  hipLaunchKernelGGL((dg3d_trace_kernel<KK>), dim3(c->E), dim3(NT3), 0, c->stream, m, c->gas, c->tab, U,     \
                     c->d_rec, RS);                                                                            \
  if (visc)                                                                                                    \
    hipLaunchKernelGGL((dg3d_residual_kernel<KK, true>), dim3(c->E), dim3(NT3), 0, c->stream, m, c->gas,      \
                       c->tab, c->flux, c->alpha, U, c->d_rec, RS, R);                                         \
  else                                                                                                         \
    hipLaunchKernelGGL((dg3d_residual_kernel<KK, false>), dim3(c->E), dim3(NT3), 0, c->stream, m, c->gas,     \
                       c->tab, c->flux, c->alpha, U, c->d_rec, RS, R);
  switch (c->K) {
    case 1: DG3_LAUNCH(1); break;
    case 2: DG3_LAUNCH(2); break;
    case 3: DG3_LAUNCH(3); break;
    default: return fail3(c, IMEX_EINVAL, "degree");
  }
#undef DG3_LAUNCH
  HIP3(c, hipGetLastError());
  return IMEX_OK;
}

const char* imex3d_last_error(const imex3d_ctx* c) { return c ? c->err.c_str() : "null context"; }

void imex3d_destroy(imex3d_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  hipFree(c->d_nbr);
  hipFree(c->d_bc);
  hipFree(c->d_h);
  hipFree(c->d_lchar);
  hipFree(c->d_rec);
  delete c;
}

}  // extern "C"
