// Device-side building blocks of the IMEX DG/HDG stage engine (gfx950).
//
// * Dual<N>: forward-mode dual numbers used to obtain the point-wise Jacobians
//   of the flux functions (the exact Newton linearisation of Sec. 4.3).
// * Flux functions of Sec. 2 (compressible Navier-Stokes, 2D), templated on the
//   scalar type so that the same code yields values and derivatives.
// * Characteristic splitting A_n^+- = P Lambda^+- P^-1 (Sec. 3.2) in closed form.
// * Basis tables for the nodal Q^k basis on Gauss-Legendre nodes with the
//   ceil((3k+1)/2)-point Gauss rule (over-integration to degree 3k, Sec. 5).
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace imex {

// --------------------------------------------------------------------------
// compile-time sizes per polynomial degree
// --------------------------------------------------------------------------
template <int K> struct Sizes {
  static constexpr int NP = K + 1;                 // 1D nodes
  static constexpr int NQ = (3 * K + 2) / 2;       // 1D quadrature points = ceil((3K+1)/2)
  static constexpr int NN = NP * NP;               // element nodes
  static constexpr int NQV = NQ * NQ;              // volume points
  static constexpr int NU = 4 * NN;                // element unknowns
  static constexpr int NF = 16 * NP;               // facet unknowns of one element (4 faces x 4 vars x NP)
  static constexpr int NFF = 4 * NP;               // unknowns of one facet
};

constexpr int MAXNP = 5;
constexpr int MAXNQ = 7;

// 1D tables of one degree (filled on the host, copied to device memory).
struct BasisTable {
  double L[MAXNQ][MAXNP];    // l_a(z_q)
  double D[MAXNQ][MAXNP];    // l_a'(z_q)
  double LE[2][MAXNP];       // l_a(-1), l_a(+1)
  double DE[2][MAXNP];       // l_a'(-1), l_a'(+1)
  double W[MAXNQ];           // Gauss weights (sum 2)
  double NW[MAXNP];          // node weights (mass matrix diagonal factors)
  double Z[MAXNQ];           // Gauss abscissae z_q on [-1, 1]
};

// --------------------------------------------------------------------------
// dual numbers
// --------------------------------------------------------------------------
template <int N> struct Dual {
  double v;
  double d[N];
  __host__ __device__ Dual() : v(0.0) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
};

template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; const double inv = 1.0 / b.v; r.v = a.v * inv;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
  return r;
}
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> __device__ inline Dual<N> operator+(double b, const Dual<N>& a) { Dual<N> r = a; r.v += b; return r; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> __device__ inline Dual<N> operator-(double b, const Dual<N>& a) { return Dual<N>(b) - a; }
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> __device__ inline Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> __device__ inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> __device__ inline Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r; r.v = ::sqrt(a.v); const double s = 0.5 / r.v;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
  return r;
}

__device__ inline double sqrt(double x) { return ::sqrt(x); }
__device__ inline float sqrt(float x) { return ::sqrtf(x); }

__device__ inline double value(double x) { return x; }
template <int N> __device__ inline double value(const Dual<N>& x) { return x.v; }
__device__ inline double value(float x) { return x; }

// |x| and max(x, 0) with the branch decided on the value (Sec. 3.2: Lambda^+- = max/min(lambda, 0))
template <class T> __device__ inline T absv(const T& x) { return value(x) >= 0.0 ? x : -x; }
template <class T> __device__ inline T posv(const T& x) { return value(x) > 0.0 ? x : T(0.0); }
template <class T> __device__ inline T negv(const T& x) { return value(x) < 0.0 ? x : T(0.0); }
template <class T> __device__ inline T maxv(const T& a, const T& b) { return value(a) >= value(b) ? a : b; }

// --------------------------------------------------------------------------
// gas constants
// --------------------------------------------------------------------------
struct Gas {
  double gamma, R, mu, Pr;
  double cv, cp, kappa, lam;    // c_v = R/(gamma-1), c_p = gamma c_v, kappa = c_p mu / Pr, lambda = -2 mu / 3
  int viscous;
  double uinf[4];
};

// --------------------------------------------------------------------------
// fluxes (Sec. 2).  F[v][d]: variable v, direction d.
// --------------------------------------------------------------------------
template <class T> struct Prim {
  T rho, u, v, E, p, theta, c, H;
};

template <class T> __device__ inline Prim<T> primitives(const T U[4], const Gas& g) {
  Prim<T> P;
  P.rho = U[0];
  const T ir = 1.0 / U[0];
  P.u = U[1] * ir;
  P.v = U[2] * ir;
  P.E = U[3] * ir;
  const T ei = P.E - 0.5 * (P.u * P.u + P.v * P.v);
  P.theta = ei * (1.0 / g.cv);
  P.p = (g.gamma - 1.0) * P.rho * ei;
  P.c = sqrt(g.gamma * (g.gamma - 1.0) * ei);
  P.H = P.E + P.p * ir;
  return P;
}

template <class T> __device__ inline void conv_flux(const T U[4], const Gas& g, T F[4][2]) {
  const Prim<T> P = primitives(U, g);
  const T rH = U[3] + P.p;
  F[0][0] = U[1];            F[0][1] = U[2];
  F[1][0] = U[1] * P.u + P.p; F[1][1] = U[1] * P.v;
  F[2][0] = U[2] * P.u;      F[2][1] = U[2] * P.v + P.p;
  F[3][0] = rH * P.u;        F[3][1] = rH * P.v;
}

// normal component of the convective flux
template <class T> __device__ inline void conv_flux_n(const T U[4], double nx, double ny, const Gas& g, T Fn[4]) {
  const Prim<T> P = primitives(U, g);
  const T un = P.u * nx + P.v * ny;
  Fn[0] = U[0] * un;
  Fn[1] = U[1] * un + P.p * nx;
  Fn[2] = U[2] * un + P.p * ny;
  Fn[3] = (U[3] + P.p) * un;
}

// Viscous flux at state W with conservative gradient G: F = K(W) G (linear in G).
// adiabatic != 0 removes the normal heat flux (q - (q.n) n).
template <class TW, class TG, class TF>
__device__ inline void visc_flux(const TW W[4], const TG G[4][2], const Gas& g, TF F[4][2],
                                 int adiabatic = 0, double nx = 0.0, double ny = 0.0) {
  const TW ir = 1.0 / W[0];
  const TW u = W[1] * ir, v = W[2] * ir, E = W[3] * ir;
  TF gu[2], gv[2], gt[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    gu[d] = (G[1][d] - u * G[0][d]) * ir;
    gv[d] = (G[2][d] - v * G[0][d]) * ir;
    const TF gE = (G[3][d] - E * G[0][d]) * ir;
    gt[d] = (gE - u * gu[d] - v * gv[d]) * (1.0 / g.cv);
  }
  const TF div = gu[0] + gv[1];
  const TF t11 = 2.0 * g.mu * gu[0] + g.lam * div;
  const TF t22 = 2.0 * g.mu * gv[1] + g.lam * div;
  const TF t12 = g.mu * (gu[1] + gv[0]);
  TF q0 = -g.kappa * gt[0], q1 = -g.kappa * gt[1];
  if (adiabatic) {
    const TF qn = q0 * nx + q1 * ny;
    q0 = q0 - qn * nx;
    q1 = q1 - qn * ny;
  }
  F[0][0] = TF(0.0); F[0][1] = TF(0.0);
  F[1][0] = t11;     F[1][1] = t12;
  F[2][0] = t12;     F[2][1] = t22;
  F[3][0] = t11 * u + t12 * v - q0;
  F[3][1] = t12 * u + t22 * v - q1;
}

// Viscous flux of the mixed form (Sec. 3.5): eps = (e11, e12, e22), phi = grad theta.
template <class TW, class TQ, class TF>
__device__ inline void visc_flux_mx(const TW W[4], const TQ eps[3], const TQ phi[2], const Gas& g, TF F[4][2]) {
  const TW ir = 1.0 / W[0];
  const TW u = W[1] * ir, v = W[2] * ir;
  const double m2 = 2.0 * g.mu;
  F[0][0] = TF(0.0); F[0][1] = TF(0.0);
  F[1][0] = m2 * eps[0]; F[1][1] = m2 * eps[1];
  F[2][0] = m2 * eps[1]; F[2][1] = m2 * eps[2];
  F[3][0] = m2 * (eps[0] * u + eps[1] * v) + g.kappa * phi[0];
  F[3][1] = m2 * (eps[1] * u + eps[2] * v) + g.kappa * phi[1];
}

// y = A_n^+(W) x (sgn = +1) or A_n^-(W) x (sgn = -1): sum_k lambda_k^+- r_k (l_k . x) with the
// closed-form right/left eigenvectors of the 2D Euler normal Jacobian (eigenvalues un-c, un, un, un+c).
template <class TW>
__device__ inline void char_apply(const TW W[4], const TW x[4], double nx, double ny, int sgn, const Gas& g, TW y[4]) {
  const Prim<TW> P = primitives(W, g);
  const double b = g.gamma - 1.0;
  const TW un = P.u * nx + P.v * ny;
  const TW ut = P.v * nx - P.u * ny;
  const TW q2 = P.u * P.u + P.v * P.v;
  const TW c = P.c;
  const TW ic2 = 1.0 / (c * c);
  // left eigenvector projections
  const TW bq = 0.5 * b * q2;
  const TW w1 = ((bq + c * un) * x[0] - (b * P.u + c * nx) * x[1] - (b * P.v + c * ny) * x[2] + b * x[3]) * (0.5 * ic2);
  const TW w2 = (1.0 - bq * ic2) * x[0] + (b * ic2) * (P.u * x[1] + P.v * x[2] - x[3]);
  const TW w3 = -ut * x[0] - ny * x[1] + nx * x[2];
  const TW w4 = ((bq - c * un) * x[0] - (b * P.u - c * nx) * x[1] - (b * P.v - c * ny) * x[2] + b * x[3]) * (0.5 * ic2);
  TW l1 = un - c, l2 = un, l4 = un + c;
  if (sgn > 0) { l1 = posv(l1); l2 = posv(l2); l4 = posv(l4); }
  else         { l1 = negv(l1); l2 = negv(l2); l4 = negv(l4); }
  const TW a1 = l1 * w1, a2 = l2 * w2, a3 = l2 * w3, a4 = l4 * w4;
  y[0] = a1 + a2 + a4;
  y[1] = a1 * (P.u - c * nx) + a2 * P.u - a3 * ny + a4 * (P.u + c * nx);
  y[2] = a1 * (P.v - c * ny) + a2 * P.v + a3 * nx + a4 * (P.v + c * ny);
  y[3] = a1 * (P.H - c * un) + a2 * (0.5 * q2) + a3 * ut + a4 * (P.H + c * un);
}

template <class T> __device__ inline T wave_speed(const T U[4], double nx, double ny, const Gas& g) {
  const Prim<T> P = primitives(U, g);
  return absv(P.u * nx + P.v * ny) + P.c;
}

// DG numerical flux (Sec. 3.3): Vijayasundaram A^+(Ubar) U + A^-(Ubar) UN, or local Lax-Friedrichs.
template <class T>
__device__ inline void dg_num_flux(const T U[4], const T UN[4], double nx, double ny, int lf, const Gas& g, T F[4]) {
  if (lf) {
    T Fa[4], Fb[4];
    conv_flux_n(U, nx, ny, g, Fa);
    conv_flux_n(UN, nx, ny, g, Fb);
    const T lam = maxv(wave_speed(U, nx, ny, g), wave_speed(UN, nx, ny, g));
#pragma unroll
    for (int v = 0; v < 4; ++v) F[v] = 0.5 * (Fa[v] + Fb[v]) + 0.5 * lam * (U[v] - UN[v]);
  } else {
    T Ub[4], ap[4], am[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Ub[v] = 0.5 * (U[v] + UN[v]);
    char_apply(Ub, U, nx, ny, +1, g, ap);
    char_apply(Ub, UN, nx, ny, -1, g, am);
#pragma unroll
    for (int v = 0; v < 4; ++v) F[v] = ap[v] + am[v];
  }
}

// HDG convective flux (eq. inviscid_numerical_flux): F_n(Uh) + S_c(Uh)(U - Uh),
// S_c = A_n^+(Uh) (flux-vector splitting) or lambda_max(Uh) I.
template <class T>
__device__ inline void hdg_num_flux(const T U[4], const T Uh[4], double nx, double ny, int lf, const Gas& g, T F[4]) {
  T Fn[4], dU[4], s[4];
  conv_flux_n(Uh, nx, ny, g, Fn);
#pragma unroll
  for (int v = 0; v < 4; ++v) dU[v] = U[v] - Uh[v];
  if (lf) {
    const T lam = wave_speed(Uh, nx, ny, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = lam * dU[v];
  } else {
    char_apply(Uh, dU, nx, ny, +1, g, s);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) F[v] = Fn[v] + s[v];
}

}  // namespace imex
