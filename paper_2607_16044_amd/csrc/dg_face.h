// Face integrand of the explicit DG-IP residual, shared by the residual kernel
// and its vector-Jacobian product.
#pragma once
#include "device_common.h"

namespace imex {

enum DGFaceKind { DGF_INTERIOR = 0, DGF_INTERFACE = 1, DGF_FARFIELD = 2 };

__device__ __forceinline__ void face_normal(int f, double& nx, double& ny) {
  nx = (f == 0) ? -1.0 : (f == 1 ? 1.0 : 0.0);
  ny = (f == 2) ? -1.0 : (f == 3 ? 1.0 : 0.0);
}

// One Gauss point of a face with outward unit normal (nx, ny) of an explicit
// element (Sec. 3.3, eq. bilinear_form_interior_sdg; far field App. B.1.1;
// interface eq. interface_bilinearform_explicit): s is the coefficient of the
// test function, gc that of its physical gradient.
//   Uo, Go  own trace and physical gradient
//   UN      neighbour trace (unused on the far field)
//   fnn     the neighbour's viscous flux F^nu . n in this element's normal
//   kind    DGF_INTERIOR (explicit neighbour): adjoint term with the own K, halved;
//           DGF_INTERFACE (implicit neighbour): adjoint term with the averaged K;
//           DGF_FARFIELD: A^+(U) U + A^-(U) U_inf, viscous terms with K(U_inf)
// Normal viscous flux of the consistency term at a face point of an explicit element:
// F^nu(U, grad U) . n, or on the far field F^nu(U_inf, grad U) . n (K at the free stream).
template <class T>
__device__ inline void dg_face_visc_n(int farfield, const T Uo[4], const T Go[4][2], double nx, double ny,
                                      const Gas& g, T fo[4]) {
  T Fv[4][2];
  if (farfield) {
    const T Ui[4] = {T(g.uinf[0]), T(g.uinf[1]), T(g.uinf[2]), T(g.uinf[3])};
    visc_flux(Ui, Go, g, Fv);
  } else {
    visc_flux(Uo, Go, g, Fv);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) fo[v] = Fv[v][0] * nx + Fv[v][1] * ny;
}

// Far-field face point (App. B.1.1) with the free-stream state Ui as an input, so that the
// same code gives the residual and, with dual numbers in Ui, its derivative in u_inf:
// s = A^+(U) U + A^-(U) Ui - fo + tau K(Ui)((U - Ui) x n) . n,  gc = -K(Ui)((U - Ui) x n),
// fo = F^nu(Ui, grad U) . n (dg_face_visc_n on the far field).
template <class T, class TI>
__device__ inline void dg_farfield_terms(const T Uo[4], const TI fo[4], const TI Ui[4], double nx, double ny,
                                         double tau, const Gas& g, TI s[4], TI gc[4][2]) {
  TI ap[4], am[4], Uc[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) Uc[v] = TI(Uo[v]);
  char_apply(Uc, Uc, nx, ny, +1, g, ap);
  char_apply(Uc, Ui, nx, ny, -1, g, am);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    s[v] = ap[v] + am[v];
    gc[v][0] = TI(0.0);
    gc[v][1] = TI(0.0);
  }
  if (!g.viscous) return;
  TI Gj[4][2], Kf[4][2];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const TI d = Uc[v] - Ui[v];
    Gj[v][0] = d * nx;
    Gj[v][1] = d * ny;
  }
  visc_flux(Ui, Gj, g, Kf);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    s[v] = s[v] - fo[v] + tau * (Kf[v][0] * nx + Kf[v][1] * ny);
    gc[v][0] = -Kf[v][0];
    gc[v][1] = -Kf[v][1];
  }
}

// The face integrand from the own trace Uo and its consistency flux fo (dg_face_visc_n):
// everything a face point needs that is not a gradient.  EULER_LF: the caller guarantees
// inviscid flow, the Lax-Friedrichs flux and no far-field face, so only that branch is
// compiled (fewer registers for the vortex workloads).
template <bool EULER_LF = false, class T>
__device__ inline void dg_face_point_fo(int kind, const T Uo[4], const T fo[4], const T UN[4], const T fnn[4],
                                        double nx, double ny, double tau, int lf, const Gas& g, T s[4],
                                        T gc[4][2]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) { gc[v][0] = T(0.0); gc[v][1] = T(0.0); }
  if (EULER_LF) {
    dg_num_flux(Uo, UN, nx, ny, 1, g, s);
    return;
  }
  if (kind != DGF_FARFIELD) {
    dg_num_flux(Uo, UN, nx, ny, lf, g, s);
    if (!g.viscous) return;
    T Gj[4][2], KU[4][2], KN[4][2];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T d = Uo[v] - UN[v];
      Gj[v][0] = d * nx;
      Gj[v][1] = d * ny;
    }
    visc_flux(Uo, Gj, g, KU);
    visc_flux(UN, Gj, g, KN);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T pen = 0.5 * ((KU[v][0] + KN[v][0]) * nx + (KU[v][1] + KN[v][1]) * ny);
      s[v] = s[v] - 0.5 * (fo[v] + fnn[v]) + tau * pen;
      if (kind == DGF_INTERFACE) {
        gc[v][0] = -0.5 * (KU[v][0] + KN[v][0]);
        gc[v][1] = -0.5 * (KU[v][1] + KN[v][1]);
      } else {
        gc[v][0] = -0.5 * KU[v][0];
        gc[v][1] = -0.5 * KU[v][1];
      }
    }
  } else {
    const T Ui[4] = {T(g.uinf[0]), T(g.uinf[1]), T(g.uinf[2]), T(g.uinf[3])};
    dg_farfield_terms(Uo, fo, Ui, nx, ny, tau, g, s, gc);
  }
}

template <class T>
__device__ inline void dg_face_point(int kind, const T Uo[4], const T Go[4][2], const T UN[4], const T fnn[4],
                                     double nx, double ny, double tau, int lf, const Gas& g, T s[4], T gc[4][2]) {
  T fo[4] = {T(0.0), T(0.0), T(0.0), T(0.0)};
  if (g.viscous) dg_face_visc_n(kind == DGF_FARFIELD, Uo, Go, nx, ny, g, fo);
  dg_face_point_fo(kind, Uo, fo, UN, fnn, nx, ny, tau, lf, g, s, gc);
}

// penalty of the face between an explicit element (measure ratio le) and its neighbour
// (ln; implicit neighbours and the far field use the element's own)
__device__ __forceinline__ double dg_tau(double alpha, int K, int kind, double le, double ln) {
  const double kk = (double)((K + 1) * (K + 1));
  return alpha * kk / ((kind == DGF_INTERIOR) ? fmin(le, ln) : le);
}

}  // namespace imex
