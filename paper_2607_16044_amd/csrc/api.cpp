// C ABI of the IMEX DG/HDG engine: context set-up, region split and the ARK
// step driver (Alg. imex_scheme_update of App. C).  All arithmetic runs in the
// kernels of dg.hip and hdg.hip; this file only builds tables, owns memory and
// sequences launches on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace imex;

namespace {

thread_local std::string g_create_error;

imex_status fail(imex_ctx* c, imex_status s, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

#define HIP_TRY(c, expr)                                                                        \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(c, IMEX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

// Gauss-Legendre points and weights on [-1,1] by Newton's method on P_n.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;                       // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

double lag(const double* nodes, int np, int a, double x) {
  double r = 1.0;
  for (int b = 0; b < np; ++b)
    if (b != a) r *= (x - nodes[b]) / (nodes[a] - nodes[b]);
  return r;
}

double dlag(const double* nodes, int np, int a, double x) {
  double s = 0.0;
  for (int c = 0; c < np; ++c) {
    if (c == a) continue;
    double t = 1.0 / (nodes[a] - nodes[c]);
    for (int b = 0; b < np; ++b)
      if (b != a && b != c) t *= (x - nodes[b]) / (nodes[a] - nodes[b]);
    s += t;
  }
  return s;
}

void build_table(int K, BasisTable& T) {
  std::memset(&T, 0, sizeof(T));
  const int np = K + 1, nq = (3 * K + 2) / 2;
  double nodes[MAXNP], nw[MAXNP], z[MAXNQ], w[MAXNQ];
  gauss_legendre(np, nodes, nw);
  gauss_legendre(nq, z, w);
  for (int a = 0; a < np; ++a) {
    T.NW[a] = nw[a];
    for (int q = 0; q < nq; ++q) {
      T.L[q][a] = lag(nodes, np, a, z[q]);
      T.D[q][a] = dlag(nodes, np, a, z[q]);
    }
    T.LE[0][a] = lag(nodes, np, a, -1.0);
    T.LE[1][a] = lag(nodes, np, a, 1.0);
    T.DE[0][a] = dlag(nodes, np, a, -1.0);
    T.DE[1][a] = dlag(nodes, np, a, 1.0);
  }
  for (int q = 0; q < nq; ++q) {
    T.W[q] = w[q];
    T.Z[q] = z[q];
  }
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) { *dst = nullptr; return hipSuccess; }
  hipError_t e = hipMalloc(dst, src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

void free_regions(imex_ctx* c) {
  for (int** p : {&c->d_im_list, &c->d_ex_list, &c->d_face_kind, &c->d_efacet, &c->d_hf_side, &c->d_hf_face,
                  &c->d_hf_elem, &c->d_win_off, &c->d_win_slot, &c->d_win_own, &c->d_sr_flags,
                  &c->d_ex_ifacet}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  Workspace& w = c->ws;
  for (double** p : {&w.rec, &w.hres, &w.Wy, &w.Hp, &w.gH, &w.gm, &w.red, &w.adj_P, &w.adj_w, &w.adj_rp, &w.adj_rm,
                     &w.adj_hp, &w.adj_hm}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  for (void** p : {&w.blk, &w.scr, &w.Kinv, &w.X, &w.Wd, &w.Wg, &w.Wc}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  if (w.hred) hipHostFree(w.hred);
  w.hred = nullptr;
  if (w.hgm) hipHostFree(w.hgm);
  w.hgm = w.hgm_dev = nullptr;
  for (double* p : w.adj_buf)
    if (p) hipFree(p);
  w.adj_buf.clear();
}

}  // namespace

// the 1D tables and Gauss rule for the other translation units (the 3D residual)
namespace imex {
void basis_table_1d(int K, BasisTable& T) { build_table(K, T); }
void gauss_legendre_rule(int n, double* x, double* w) { gauss_legendre(n, x, w); }
}  // namespace imex

void imex_ctx::drop_graphs() {
  for (StageGraph& g : sg) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.key.clear();
  }
  for (auto& kv : gm_graphs)
    if (kv.second) hipGraphExecDestroy(kv.second);
  gm_graphs.clear();
}

int imex_ctx::timer_begin(int tag) {
  if (capturing || !((timer_mask >> tag) & 1u)) return -1;
  hipEvent_t a, b;
  if (ev_free.size() >= 2) {
    a = ev_free.back(); ev_free.pop_back();
    b = ev_free.back(); ev_free.pop_back();
  } else {
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); return -1; }
  }
  hipEventRecord(a, stream);
  ev_pending.push_back({tag, a, b});
  return (int)ev_pending.size() - 1;
}

void imex_ctx::timer_end(int idx) {
  if (idx < 0 || idx >= (int)ev_pending.size()) return;
  hipEventRecord(ev_pending[idx].b, stream);
}

void imex_ctx::timers_resolve() {
  for (const Pending& p : ev_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      tm_ms[p.tag] += ms;
      tm_n[p.tag] += 1;
    }
    ev_free.push_back(p.a);
    ev_free.push_back(p.b);
  }
  ev_pending.clear();
}

extern "C" {

const char* imex_status_str(imex_status s) {
  switch (s) {
    case IMEX_OK: return "ok";
    case IMEX_EINVAL: return "invalid argument";
    case IMEX_ENOMEM: return "out of device memory";
    case IMEX_EDEVICE: return "HIP error";
    case IMEX_ENOCONV: return "Newton did not converge";
    case IMEX_ENONFINITE: return "non-finite value";
    case IMEX_ENOTIMPL: return "not implemented";
    case IMEX_ESTATE: return "invalid call order";
  }
  return "unknown status";
}

const char* imex_last_error(const imex_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

static imex_status check_mesh(const imex_mesh_desc* mesh) {
  if (mesh->nx < 1 || mesh->ny < 1 || !mesh->xgrid || !mesh->ygrid)
    return fail(nullptr, IMEX_EINVAL, "mesh needs nx, ny >= 1 and both grids");
  if (mesh->degree < 1 || mesh->degree > 4) return fail(nullptr, IMEX_EINVAL, "degree must be in 1..4");
  for (int a = 0; a < 2; ++a) {
    const bool p0 = mesh->bc[2 * a] == IMEX_BC_PERIODIC, p1 = mesh->bc[2 * a + 1] == IMEX_BC_PERIODIC;
    if (p0 != p1) return fail(nullptr, IMEX_EINVAL, "periodic boundaries must pair");
  }
  for (int s = 0; s < 4; ++s)
    if (mesh->bc[s] < 0 || mesh->bc[s] > 2) return fail(nullptr, IMEX_EINVAL, "unknown boundary type");
  for (int i = 0; i < mesh->nx; ++i)
    if (!(mesh->xgrid[i + 1] > mesh->xgrid[i])) return fail(nullptr, IMEX_EINVAL, "xgrid not increasing");
  for (int j = 0; j < mesh->ny; ++j)
    if (!(mesh->ygrid[j + 1] > mesh->ygrid[j])) return fail(nullptr, IMEX_EINVAL, "ygrid not increasing");
  return IMEX_OK;
}

// One context over n structured meshes of the same degree (their disjoint union).
static imex_status create_ctx(int n, const imex_mesh_desc* meshes, const double* dt_scale,
                              const imex_physics* phys, const imex_options* opt, void* stream, imex_ctx** out) {
  if (!meshes || !phys || !opt || !out || n < 1) return fail(nullptr, IMEX_EINVAL, "null argument or no mesh");
  *out = nullptr;
  long long Etot = 0;
  for (int k = 0; k < n; ++k) {
    imex_status st = check_mesh(&meshes[k]);
    if (st != IMEX_OK) return st;
    if (meshes[k].degree != meshes[0].degree) return fail(nullptr, IMEX_EINVAL, "all meshes need the same degree");
    if (dt_scale && !(dt_scale[k] > 0.0)) return fail(nullptr, IMEX_EINVAL, "time-step scales must be positive");
    Etot += (long long)meshes[k].nx * meshes[k].ny;
  }
  if (Etot > (1LL << 28)) return fail(nullptr, IMEX_EINVAL, "too many elements");
  if (!(phys->gamma > 1.0) || !(phys->R > 0.0) || phys->mu < 0.0 || !(phys->Pr > 0.0))
    return fail(nullptr, IMEX_EINVAL, "bad gas constants");
  if (opt->hdg_variant != IMEX_HDG_IP && opt->hdg_variant != IMEX_HDG_MX)
    return fail(nullptr, IMEX_EINVAL, "hdg_variant");
  if (opt->precision != IMEX_FP64 && opt->precision != IMEX_FP32_REFINE)
    return fail(nullptr, IMEX_EINVAL, "precision");
  if (opt->newton_maxit < 1 || opt->gmres_restart < 1 || opt->gmres_restart > 64 || opt->gmres_maxit < 1 ||
      !(opt->newton_rtol > 0.0) || !(opt->gmres_rtol > 0.0) || opt->newton_simplified < 0 ||
      opt->newton_simplified > 2 || opt->gmres_forcing < 0 || opt->gmres_forcing > 3)
    return fail(nullptr, IMEX_EINVAL, "solver options");

  imex_ctx* c = new (std::nothrow) imex_ctx();
  if (!c) return fail(nullptr, IMEX_ENOMEM, "host allocation");
  hipGetDevice(&c->device);
  // the static scratch of imex_dg_residual_noalloc: its device address, once per device
  // (a failure here is reported by that entry point, which cannot run without it)
  static_scratch_init(c->device);
  c->stream = static_cast<hipStream_t>(stream);
  c->E = (int)Etot;
  c->K = meshes[0].degree;
  c->NP = c->K + 1;
  c->NQ = (3 * c->K + 2) / 2;
  c->NN = c->NP * c->NP;
  c->opt = *opt;
  Gas& g = c->gas;
  g.gamma = phys->gamma;
  g.R = phys->R;
  g.mu = phys->viscous ? phys->mu : 0.0;
  g.Pr = phys->Pr;
  g.cv = g.R / (g.gamma - 1.0);
  g.cp = g.gamma * g.cv;
  g.kappa = g.cp * g.mu / g.Pr;
  g.lam = -2.0 * g.mu / 3.0;
  g.viscous = phys->viscous ? 1 : 0;
  for (int v = 0; v < 4; ++v) g.uinf[v] = phys->u_inf[v];
  build_table(c->K, c->tab);

  // geometry and neighbours, instance by instance
  const int E = c->E;
  std::vector<double> hx(E), hy(E), dts(E, 1.0), xy0(2 * (size_t)E);
  c->nbr.assign(4 * E, -1);
  c->bcf.assign(4 * E, -1);
  int off = 0;
  for (int k = 0; k < n; ++k) {
    const imex_mesh_desc* mesh = &meshes[k];
    Inst in;
    in.nx = mesh->nx;
    in.ny = mesh->ny;
    in.e_off = off;
    in.dt_scale = dt_scale ? dt_scale[k] : 1.0;
    std::memcpy(in.bc, mesh->bc, sizeof(in.bc));
    in.xg.assign(mesh->xgrid, mesh->xgrid + in.nx + 1);
    in.yg.assign(mesh->ygrid, mesh->ygrid + in.ny + 1);
    const int nx = in.nx, ny = in.ny;
    const bool px = mesh->bc[0] == IMEX_BC_PERIODIC, py = mesh->bc[2] == IMEX_BC_PERIODIC;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int e = off + i + nx * j;
        hx[e] = in.xg[i + 1] - in.xg[i];
        hy[e] = in.yg[j + 1] - in.yg[j];
        xy0[2 * e] = in.xg[i];
        xy0[2 * e + 1] = in.yg[j];
        dts[e] = in.dt_scale;
        const int ci[4] = {i - 1, i + 1, i, i};
        const int cj[4] = {j, j, j - 1, j + 1};
        for (int f = 0; f < 4; ++f) {
          int a = ci[f], b = cj[f];
          const bool inside = a >= 0 && a < nx && b >= 0 && b < ny;
          if (!inside) {
            if (f < 2 && px) a = (a + nx) % nx;
            else if (f >= 2 && py) b = (b + ny) % ny;
            else { c->bcf[4 * e + f] = mesh->bc[f]; continue; }
          }
          c->nbr[4 * e + f] = off + a + nx * b;
        }
      }
    off += nx * ny;
    c->inst.push_back(std::move(in));
  }
  c->imp.assign(E, 0);
  c->err.clear();
  hipStream_t s = c->stream;
  hipError_t he = hipSuccess;
  if ((he = upload(&c->d_hx, hx, s)) != hipSuccess || (he = upload(&c->d_hy, hy, s)) != hipSuccess ||
      (he = upload(&c->d_xy0, xy0, s)) != hipSuccess ||
      (he = upload(&c->d_nbr, c->nbr, s)) != hipSuccess || (he = upload(&c->d_bcf, c->bcf, s)) != hipSuccess ||
      (he = upload(&c->d_imp, c->imp, s)) != hipSuccess || (dt_scale && (he = upload(&c->d_dts, dts, s)) != hipSuccess)) {
    imex_destroy(c);
    return fail(nullptr, IMEX_ENOMEM, std::string("device tables: ") + hipGetErrorString(he));
  }
  he = hipMalloc(&c->d_tab, sizeof(BasisTable));
  if (he == hipSuccess) he = hipMemcpyAsync(c->d_tab, &c->tab, sizeof(BasisTable), hipMemcpyHostToDevice, s);
  // element-sized work arrays
  const size_t es = (size_t)E * 4 * c->NN;
  Workspace& w = c->ws;
  if (he == hipSuccess) he = hipMalloc(&w.trace, (size_t)E * 4 * c->NQ * 8 * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&w.Q, (size_t)E * 5 * c->NN * sizeof(double));
  if (he == hipSuccess) he = hipMemsetAsync(w.Q, 0, (size_t)E * 5 * c->NN * sizeof(double), s);
  for (int r = 0; r < 8 && he == hipSuccess; ++r) he = hipMalloc(&w.Rstage[r], es * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&w.Un, es * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&w.Y, es * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&w.rhs, es * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&w.Yp, es * sizeof(double));
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    imex_destroy(c);
    return fail(nullptr, IMEX_ENOMEM, std::string("workspace: ") + hipGetErrorString(he));
  }
  w.bytes = (size_t)E * 4 * c->NQ * 8 * 8 + (size_t)E * 5 * c->NN * 8 + 12 * es * 8;
  *out = c;
  return IMEX_OK;
}

imex_status imex_create(const imex_mesh_desc* mesh, const imex_physics* phys, const imex_options* opt, void* stream,
                        imex_ctx** out) {
  return create_ctx(1, mesh, nullptr, phys, opt, stream, out);
}

imex_status imex_create_batch(int n_inst, const imex_mesh_desc* meshes, const double* dt_scale,
                              const imex_physics* phys, const imex_options* opt, void* stream, imex_ctx** out) {
  return create_ctx(n_inst, meshes, dt_scale, phys, opt, stream, out);
}

imex_status imex_set_regions(imex_ctx* c, const unsigned char* flag) {
  if (!c || !flag) return fail(c, IMEX_EINVAL, "null argument");
  const int E = c->E;
  // validate before anything in the context changes
  for (int e = 0; e < E; ++e)
    if (!flag[e])
      for (int f = 0; f < 4; ++f)
        if (c->nbr[4 * e + f] < 0 && c->bcf[4 * e + f] == IMEX_BC_WALL)
          return fail(c, IMEX_EINVAL, "adiabatic walls are supported on implicit elements only");
  // the workspaces below are freed and reallocated: finish queued work and drop every
  // captured graph (their kernel arguments point into the old workspaces).  The context
  // counts as unconfigured until the new regions are complete.
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->drop_graphs();
  c->regions_set = false;
  c->prec_valid = false;
  c->prec_fresh = false;
  c->newton_q2 = 0.0;
  for (int& g : c->gm_hist) g = 0;
  c->imp.assign(flag, flag + E);
  for (int e = 0; e < E; ++e) c->imp[e] = c->imp[e] ? 1 : 0;
  c->im_list.clear();
  c->ex_list.clear();
  for (int e = 0; e < E; ++e) (c->imp[e] ? c->im_list : c->ex_list).push_back(e);
  c->n_im = (int)c->im_list.size();
  c->n_ex = (int)c->ex_list.size();
  c->dg_farfield = false;
  for (int e : c->ex_list)
    for (int f = 0; f < 4; ++f)
      if (c->nbr[4 * e + f] < 0 && c->bcf[4 * e + f] == IMEX_BC_FARFIELD) c->dg_farfield = true;
  std::vector<int> im_pos(E, -1);
  for (int p = 0; p < c->n_im; ++p) im_pos[c->im_list[p]] = p;
  // HDG facets of each instance: vertical (x = x_i) then horizontal (y = y_j), keeping those
  // touching an implicit element; ids continue over the instances
  c->hf_side.clear();
  c->hf_face.clear();
  c->hf_elem.clear();
  c->efacet.assign(4 * c->n_im, -1);
  auto add = [&](int eL, int fL, int eR, int fR) {
    const bool keep = (eL >= 0 && c->imp[eL]) || (eR >= 0 && c->imp[eR]);
    if (!keep) return;
    const int id = (int)(c->hf_side.size() / 2);
    const int ee[2] = {eL, eR}, ff[2] = {fL, fR};
    for (int s = 0; s < 2; ++s) {
      const int e = ee[s];
      c->hf_elem.push_back(e);
      c->hf_face.push_back(ff[s]);
      c->hf_side.push_back(e >= 0 ? im_pos[e] : -1);
      if (e >= 0 && im_pos[e] >= 0) c->efacet[4 * im_pos[e] + ff[s]] = id;
    }
  };
  std::vector<int> hf_base;
  for (const Inst& in : c->inst) {
    hf_base.push_back((int)(c->hf_side.size() / 2));
    const int nx = in.nx, ny = in.ny, o = in.e_off;
    const bool px = in.bc[0] == IMEX_BC_PERIODIC, py = in.bc[2] == IMEX_BC_PERIODIC;
    const int nvx = px ? nx : nx + 1, nhy = py ? ny : ny + 1;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nvx; ++i) {
        const int eR = i < nx ? o + i + nx * j : -1;
        const int eL = i > 0 ? o + (i - 1) + nx * j : (px ? o + (nx - 1) + nx * j : -1);
        add(eL, 1, eR, 0);
      }
    for (int j = 0; j < nhy; ++j)
      for (int i = 0; i < nx; ++i) {
        const int eR = j < ny ? o + i + nx * j : -1;
        const int eL = j > 0 ? o + i + nx * (j - 1) : (py ? o + i + nx * (ny - 1) : -1);
        add(eL, 3, eR, 2);
      }
  }
  c->n_hf = (int)(c->hf_side.size() / 2);
  // Two-column Schwarz windows for the facet preconditioner, per instance.  Window w covers
  // element columns c0 = w and c1 = w + 1 (wrapping when periodic in x); its unknowns are the
  // HDG facets of those columns, grouped in super-rows r (element rows) with slots
  // [H(c0, r), H(c1, r), V(x_c0, r), V(x_c0+1, r), V(x_c1+1, r)], plus a last super-row
  // holding the top horizontal facets.  A window writes only the facets it owns (column
  // c0's horizontal facets and left vertical facets; the last window of a non-periodic
  // mesh also owns its second column), so every facet is written exactly once.
  c->win_off.assign(1, 0);
  c->win_slot.clear();
  c->win_own.clear();
  c->n_win = 0;
  std::vector<int> owned(c->n_hf, 0);
  for (size_t k = 0; k < c->inst.size(); ++k) {
    const Inst& in = c->inst[k];
    const int nx = in.nx, ny = in.ny, o = in.e_off;
    const bool px = in.bc[0] == IMEX_BC_PERIODIC, py = in.bc[2] == IMEX_BC_PERIODIC;
    const int nvx = px ? nx : nx + 1, nhy = py ? ny : ny + 1;
    std::vector<int> vid((nx + 1) * ny, -1), hid(nx * (ny + 1), -1);
    int id = hf_base[k];
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nvx; ++i) {
        const int eR = i < nx ? o + i + nx * j : -1;
        const int eL = i > 0 ? o + (i - 1) + nx * j : (px ? o + (nx - 1) + nx * j : -1);
        if ((eL >= 0 && c->imp[eL]) || (eR >= 0 && c->imp[eR])) vid[i + (nx + 1) * j] = id++;
      }
    for (int j = 0; j < nhy; ++j)
      for (int i = 0; i < nx; ++i) {
        const int eR = j < ny ? o + i + nx * j : -1;
        const int eL = j > 0 ? o + i + nx * (j - 1) : (py ? o + i + nx * (ny - 1) : -1);
        if ((eL >= 0 && c->imp[eL]) || (eR >= 0 && c->imp[eR])) hid[i + nx * j] = id++;
      }
    auto V = [&](int xi, int j) -> int {          // vertical facet at x_xi, row j
      if (px) xi = ((xi % nx) + nx) % nx;
      if (xi < 0 || xi > nx || j < 0 || j >= ny) return -1;
      return vid[xi + (nx + 1) * j];
    };
    auto H = [&](int i, int j) -> int {           // horizontal facet of column i at y_j
      if (i < 0 || i >= nx || j < 0) return -1;
      if (py) j = j % ny;
      if (j > (py ? ny - 1 : ny)) return -1;
      return hid[i + nx * j];
    };
    const int nwin = (nx == 1) ? 1 : (px ? nx : nx - 1);
    for (int w = 0; w < nwin; ++w) {
      const int c0 = w;
      const int c1 = (nx == 1) ? -1 : (px ? (w + 1) % nx : w + 1);
      const bool last = !px && (w == nwin - 1);
      int rlo = ny, rhi = -1;
      for (int j = 0; j < ny; ++j)
        for (int col : {c0, c1})
          if (col >= 0 && c->imp[o + col + nx * j]) { rlo = std::min(rlo, j); rhi = std::max(rhi, j); }
      if (rhi < 0) { c->win_off.push_back((int)(c->win_slot.size() / 5)); continue; }
      for (int r = rlo; r <= rhi + 1; ++r) {
        int f[5] = {H(c0, r), c1 >= 0 ? H(c1, r) : -1, -1, -1, -1};
        if (r <= rhi) {
          f[2] = V(c0, r);
          f[3] = V(c0 + 1, r);
          f[4] = c1 >= 0 ? V(c1 + 1, r) : -1;
        }
        if (py && r == rhi + 1 && rhi == ny - 1 && rlo == 0) { f[0] = -1; f[1] = -1; }   // wrapped top row
        for (int a = 0; a < 5; ++a)
          for (int b2 = 0; b2 < a; ++b2)
            if (f[a] >= 0 && f[a] == f[b2]) f[a] = -1;
        for (int a = 0; a < 5; ++a) {
          const bool own = f[a] >= 0 && (a == 0 || a == 2 || last || c1 < 0) && !owned[f[a]];
          if (own) owned[f[a]] = 1;
          c->win_slot.push_back(f[a]);
          c->win_own.push_back(own ? 1 : 0);
        }
      }
      c->win_off.push_back((int)(c->win_slot.size() / 5));
    }
    c->n_win += nwin;
  }
  c->n_superrows = (int)(c->win_slot.size() / 5);
  // facets of implicit regions with ragged column extents: first occurrence owns them
  for (size_t q = 0; q < c->win_slot.size(); ++q) {
    const int f = c->win_slot[q];
    if (f >= 0 && !owned[f]) { owned[f] = 1; c->win_own[q] = 1; }
  }
  for (int f = 0; f < c->n_hf; ++f)
    if (!owned[f]) return fail(c, IMEX_EINVAL, "facet preconditioner windows do not cover every facet");
  // per super-row: bit 0 = has a predecessor, bit 1 = has a successor in its window
  c->sr_flags.assign(c->n_superrows, 0);
  for (int w = 0; w < c->n_win; ++w)
    for (int g = c->win_off[w]; g < c->win_off[w + 1]; ++g)
      c->sr_flags[g] = (g > c->win_off[w] ? 1 : 0) | (g + 1 < c->win_off[w + 1] ? 2 : 0);
  c->face_kind.assign(4 * c->n_im, 0);
  for (int p = 0; p < c->n_im; ++p) {
    const int e = c->im_list[p];
    for (int f = 0; f < 4; ++f) {
      const int nb = c->nbr[4 * e + f];
      int k;
      if (nb >= 0) k = c->imp[nb] ? FK_INTERIOR : FK_INTERFACE;
      else k = (c->bcf[4 * e + f] == IMEX_BC_FARFIELD) ? FK_FARFIELD : FK_WALL;
      c->face_kind[4 * p + f] = k;
    }
  }
  // interface facet across each face of an explicit element (adjoint of the interface rows)
  c->ex_ifacet.assign(4 * (size_t)E, -1);
  for (int e : c->ex_list)
    for (int f = 0; f < 4; ++f) {
      const int nb = c->nbr[4 * e + f];
      if (nb >= 0 && c->imp[nb]) c->ex_ifacet[4 * e + f] = c->efacet[4 * im_pos[nb] + (f ^ 1)];
    }
  free_regions(c);
  hipStream_t s = c->stream;
  hipError_t he = hipMemcpyAsync(c->d_imp, c->imp.data(), E, hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = upload(&c->d_im_list, c->im_list, s);
  if (he == hipSuccess) he = upload(&c->d_ex_list, c->ex_list, s);
  if (he == hipSuccess) he = upload(&c->d_face_kind, c->face_kind, s);
  if (he == hipSuccess) he = upload(&c->d_efacet, c->efacet, s);
  if (he == hipSuccess) he = upload(&c->d_hf_side, c->hf_side, s);
  if (he == hipSuccess) he = upload(&c->d_hf_face, c->hf_face, s);
  if (he == hipSuccess) he = upload(&c->d_hf_elem, c->hf_elem, s);
  if (he == hipSuccess) he = upload(&c->d_win_off, c->win_off, s);
  if (he == hipSuccess) he = upload(&c->d_win_slot, c->win_slot, s);
  if (he == hipSuccess) he = upload(&c->d_win_own, c->win_own, s);
  if (he == hipSuccess) he = upload(&c->d_sr_flags, c->sr_flags, s);
  if (he == hipSuccess) he = upload(&c->d_ex_ifacet, c->ex_ifacet, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return fail(c, IMEX_ENOMEM, std::string("region tables: ") + hipGetErrorString(he));
  imex_status st = hdg_alloc(c);
  if (st != IMEX_OK) return st;
  c->regions_set = true;
  return IMEX_OK;
}

imex_status imex_query_sizes(const imex_ctx* c, long long out[8]) {
  if (!c || !out) return IMEX_EINVAL;
  out[0] = c->E;
  out[1] = c->n_im;
  out[2] = c->regions_set ? c->n_ex : c->E;
  out[3] = c->NN;
  out[4] = c->n_hf;
  out[5] = 4 * c->NP;
  out[6] = c->NQ;
  out[7] = (long long)c->ws.bytes;
  return IMEX_OK;
}

imex_status imex_node_coords(const imex_ctx* c, double* x, double* y) {
  if (!c || !x || !y) return IMEX_EINVAL;
  double nodes[MAXNP], nw[MAXNP];
  gauss_legendre(c->NP, nodes, nw);
  for (const Inst& in : c->inst)
    for (int j = 0; j < in.ny; ++j)
      for (int i = 0; i < in.nx; ++i) {
        const int e = in.e_off + i + in.nx * j;
        const double hx = in.xg[i + 1] - in.xg[i], hy = in.yg[j + 1] - in.yg[j];
        for (int n = 0; n < c->NN; ++n) {
          x[(size_t)e * c->NN + n] = in.xg[i] + 0.5 * (nodes[n % c->NP] + 1.0) * hx;
          y[(size_t)e * c->NN + n] = in.yg[j] + 0.5 * (nodes[n / c->NP] + 1.0) * hy;
        }
      }
  return IMEX_OK;
}

imex_status imex_init_facets(imex_ctx* c, const double* U, double* Uhat) {
  if (!c || !U || !Uhat) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (c->n_hf == 0) return IMEX_OK;
  HIP_TRY(c, launch_init_facets(c, U, Uhat));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

imex_status imex_vjp_init_facets(imex_ctx* c, const double* Uhatbar, double* Ubar) {
  if (!c || !Uhatbar || !Ubar) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (c->n_hf == 0) return IMEX_OK;
  HIP_TRY(c, launch_init_facets_vjp(c, Uhatbar, Ubar));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

imex_status imex_wall_shear(imex_ctx* c, const double* U, const double* Uhat, double* J) {
  if (!c || !U || !J) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  *J = 0.0;
  if (c->n_im == 0) return IMEX_OK;
  if (!Uhat) return fail(c, IMEX_EINVAL, "null argument");
  if (c->opt.hdg_variant != IMEX_HDG_MX || !c->gas.viscous)
    return fail(c, IMEX_ENOTIMPL, "the wall shear is taken from the HDG-MX mixed variables");
  Workspace& w = c->ws;
  HIP_TRY(c, vjp_alloc(c));
  HIP_TRY(c, launch_lift_mixed(c, U, Uhat, w.vjp_q));
  HIP_TRY(c, launch_wall_shear(c, w.vjp_q, w.red));
  HIP_TRY(c, hipMemcpyAsync(w.hred, w.red, sizeof(double) * c->n_im, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int p = 0; p < c->n_im; ++p) s += w.hred[p];
  *J = s;
  return IMEX_OK;
}

imex_status imex_vjp_wall_shear(imex_ctx* c, const double* U, const double* Uhat, double Jbar, double* Ubar,
                                double* Uhatbar) {
  if (!c || !U || !Ubar) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (c->n_im == 0) return IMEX_OK;
  if (!Uhat || !Uhatbar) return fail(c, IMEX_EINVAL, "null argument");
  if (c->opt.hdg_variant != IMEX_HDG_MX || !c->gas.viscous)
    return fail(c, IMEX_ENOTIMPL, "the wall shear is taken from the HDG-MX mixed variables");
  Workspace& w = c->ws;
  HIP_TRY(c, vjp_alloc(c));
  HIP_TRY(c, hipMemsetAsync(w.vjp_qb, 0, sizeof(double) * (size_t)c->E * 5 * c->NN, c->stream));
  HIP_TRY(c, launch_wall_shear_qbar(c, 2.0 * c->gas.mu * Jbar, w.vjp_qb));
  HIP_TRY(c, launch_lift_vjp(c, U, Uhat, w.vjp_qb, Ubar, w.vjp_hb, Uhatbar));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

static imex_status dg_residual_async(imex_ctx* c, const double* U, const double* Uhat, double* R) {
  const bool mx = c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous && c->n_im > 0;
  if (mx && Uhat) HIP_TRY(c, launch_lift_mixed(c, U, Uhat, c->ws.Q));
  HIP_TRY(c, launch_dg_trace(c, U, mx ? c->ws.Q : nullptr, c->ws.trace));
  HIP_TRY(c, hipMemsetAsync(R, 0, (size_t)c->E * 4 * c->NN * sizeof(double), c->stream));
  HIP_TRY(c, launch_dg_residual(c, U, c->ws.trace, R));
  return IMEX_OK;
}

extern "C++" {
// Run body() on the context's stream, or, with graphs enabled, replay the graph of
// slot captured from it (captured again when key changes: dt, coefficients).
template <class F>
static imex_status run_captured(imex_ctx* c, int slot, const std::vector<double>& key, F&& body) {
  if (!c->use_graphs) return body();
  imex_ctx::StageGraph& g = c->sg[slot];
  if (!g.exec || g.key != key) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    hipStream_t orig = c->stream;
    HIP_TRY(c, hipStreamSynchronize(orig));
    HIP_TRY(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeRelaxed));
    c->stream = c->gstream;
    c->capturing = true;
    imex_status st = body();
    c->capturing = false;
    c->stream = orig;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->gstream, &graph);
    if (st != IMEX_OK) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    if (ec != hipSuccess) return fail(c, IMEX_EDEVICE, std::string("stream capture: ") + hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      return fail(c, IMEX_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    g.key = key;
  }
  HIP_TRY(c, hipGraphLaunch(g.exec, c->stream));
  return IMEX_OK;
}
}  // extern "C++"

imex_status imex_dg_residual(imex_ctx* c, const double* U, const double* Uhat, double* R) {
  if (!c || !U || !R) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  imex_status st = dg_residual_async(c, U, Uhat, R);
  if (st != IMEX_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

imex_status imex_set_mms_source(imex_ctx* c, const double params[3], double t0, int on) {
  if (!c || (on && !params)) return fail(c, IMEX_EINVAL, "null argument");
  if (on && !(std::isfinite(params[0]) && std::isfinite(params[1]) && std::isfinite(params[2]) && std::isfinite(t0)))
    return fail(c, IMEX_EINVAL, "non-finite source parameters");
  if (on && c->d_dts) return fail(c, IMEX_EINVAL, "the source needs one time step for the whole context");
  if (on && !c->d_src) {
    HIP_TRY(c, hipMalloc(&c->d_src, sizeof(double) * (size_t)c->E * 4 * c->NN));
    c->ws.bytes += sizeof(double) * (size_t)c->E * 4 * c->NN;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->drop_graphs();                          // the captured stage sequences change
  c->mms_on = on != 0;
  if (on)
    for (int i = 0; i < 3; ++i) c->mms[i] = params[i];
  c->t_now = t0;
  return IMEX_OK;
}

imex_status imex_mms_load(imex_ctx* c, double t, double* b) {
  if (!c || !b) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->mms_on) return fail(c, IMEX_ESTATE, "imex_set_mms_source first");
  HIP_TRY(c, launch_mms_load(c, t, b));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

imex_status imex_dg_residual_noalloc(imex_ctx* c, const double* U, const double* Uhat, double* R) {
  if (!c || !U || !R) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  const bool mx = c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous && c->n_im > 0;
  if (mx && !Uhat) return fail(c, IMEX_EINVAL, "Uhat required with an HDG-MX region");
  const size_t n_trace = (size_t)c->E * 4 * c->NQ * 8, n_q = mx ? (size_t)c->E * 5 * c->NN : 0;
  if (n_trace + n_q > STATIC_SCRATCH_DOUBLES)
    return fail(c, IMEX_EINVAL, "mesh too large for the static scratch (" + std::to_string(n_trace + n_q) +
                                    " > " + std::to_string(STATIC_SCRATCH_DOUBLES) + " doubles)");
  double* base = static_scratch(c->device);
  if (!base) return fail(c, IMEX_EDEVICE, "static scratch address not resolved on this device");
  double* trace = base;
  double* Q = base + n_trace;
  if (mx) HIP_TRY(c, launch_lift_mixed(c, U, Uhat, Q));
  HIP_TRY(c, launch_dg_trace(c, U, mx ? Q : nullptr, trace));
  HIP_TRY(c, launch_fill_zero(c, R, (size_t)c->E * 4 * c->NN));
  HIP_TRY(c, launch_dg_residual(c, U, trace, R));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

imex_status imex_implicit_stage_solve(imex_ctx* c, double dt_a, const double* rhs, double* U, double* Uhat,
                                      double* R_out, imex_stats* st) {
  if (!c || !rhs || !U || !Uhat) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set || c->n_im == 0) return fail(c, IMEX_ESTATE, "no implicit region");
  if (!(dt_a > 0.0)) return fail(c, IMEX_EINVAL, "dt_aii must be positive");
  if (st) std::memset(st, 0, sizeof(*st));
  return hdg_stage_solve(c, dt_a, rhs, U, Uhat, R_out, st);
}

imex_status imex_local_system(imex_ctx* c, double dt_a, const double* rhs, const double* U, const double* Uhat,
                              double* f, double* h, double* K, double* C, double* D, double* E) {
  if (!c || !rhs || !U || !Uhat || !f || !h || !K || !C || !D || !E) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set || c->n_im == 0) return fail(c, IMEX_ESTATE, "no implicit region");
  return hdg_local_system(c, dt_a, rhs, U, Uhat, f, h, K, C, D, E);
}

}  // extern "C"

// Checks an ARK pair before any work: s in 1..3, a strictly lower triangular explicit
// tableau, and the fsal / stiffly_accurate flags equal to what the coefficients say
// (fsal: be is the last row of Ae; stiffly accurate: bi is the last row of Ai; Sec. 4.2.2).
// Implicit tableaux that are not stiffly accurate are not implemented with an implicit
// region (the final implicit update would need R^HDG of every stage at U_{n+1}).
static imex_status check_tableau(imex_ctx* c, const imex_tableau* tab, double dt) {
  if (tab->s < 1 || tab->s > 3 || !(dt > 0.0)) return fail(c, IMEX_EINVAL, "tableau stages or dt");
  const int s = tab->s;
  for (int i = 0; i <= s; ++i)
    for (int j = i; j <= s; ++j)
      if (tab->Ae[4 * i + j] != 0.0) return fail(c, IMEX_EINVAL, "explicit tableau not strictly lower triangular");
  for (int i = 0; i < s; ++i)
    for (int j = i + 1; j < s; ++j)
      if (tab->Ai[3 * i + j] != 0.0) return fail(c, IMEX_EINVAL, "implicit tableau not lower triangular");
  bool fsal = true, sa = true;
  for (int j = 0; j <= s; ++j) fsal = fsal && tab->be[j] == tab->Ae[4 * s + j];
  for (int j = 0; j < s; ++j) sa = sa && tab->bi[j] == tab->Ai[3 * (s - 1) + j];
  if ((tab->fsal != 0) != fsal) return fail(c, IMEX_EINVAL, "fsal flag disagrees with be and the last row of Ae");
  if ((tab->stiffly_accurate != 0) != sa)
    return fail(c, IMEX_EINVAL, "stiffly_accurate flag disagrees with bi and the last row of Ai");
  if (c->n_im > 0 && !sa) return fail(c, IMEX_ENOTIMPL, "implicit tableaux that are not stiffly accurate");
  return IMEX_OK;
}

// Stage data recorded by a step for its reverse mode: Ydg[i] = state entering the
// explicit residual of stage i+1 (Ydg[s]: the final residual, not FSAL); Ysol[i],
// Hsol[i] = stage state and facet state after the implicit solve of stage i+1.
struct ArkTape {
  double* Ydg[4] = {};
  double* Ysol[3] = {};
  double* Hsol[3] = {};
};

static imex_status ark_step_impl(imex_ctx* c, const imex_tableau* tab, double dt, double* U, double* Uhat,
                                 imex_stats* st, const ArkTape* tape);

extern "C" {

imex_status imex_ark_step(imex_ctx* c, const imex_tableau* tab, double dt, double* U, double* Uhat, imex_stats* st) {
  return ark_step_impl(c, tab, dt, U, Uhat, st, nullptr);
}

}  // extern "C"

static imex_status ark_step_impl(imex_ctx* c, const imex_tableau* tab, double dt, double* U, double* Uhat,
                                 imex_stats* st, const ArkTape* tape) {
  if (!c || !tab || !U) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (c->n_im > 0 && !Uhat) return fail(c, IMEX_EINVAL, "Uhat required with an implicit region");
  if (imex_status ts = check_tableau(c, tab, dt); ts != IMEX_OK) return ts;
  if (st) std::memset(st, 0, sizeof(*st));
  Workspace& w = c->ws;
  const int s = tab->s;
  const size_t n = (size_t)c->E * 4 * c->NN;
  hipStream_t hs = c->stream;
  const bool mx = c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous && c->n_im > 0;
  double* Rdg[4] = {w.Rstage[0], w.Rstage[1], w.Rstage[2], w.Rstage[3]};
  double* Rhdg[3] = {w.Rstage[4], w.Rstage[5], w.Rstage[6]};
  HIP_TRY(c, hipMemcpyAsync(w.Un, U, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  HIP_TRY(c, hipMemcpyAsync(w.Y, U, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  if (c->n_im > 0) {
    HIP_TRY(c, hipMemcpyAsync(w.Yp, U, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
    HIP_TRY(c, hipMemcpyAsync(w.Hp, Uhat, (size_t)c->n_hf * 4 * c->NP * sizeof(double), hipMemcpyDeviceToDevice, hs));
  }
  // implicit stage times c_i = sum_j a_ij (c_0 = 0); explicit stage times cbar_i = row sums of Ae
  double ci[4] = {0.0, 0.0, 0.0, 0.0}, ce[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 1; i <= s; ++i)
    for (int j = 0; j < i; ++j) ci[i] += tab->Ai[3 * (i - 1) + j];
  for (int i = 0; i <= s; ++i)
    for (int j = 0; j < i; ++j) ce[i] += tab->Ae[4 * i + j];
  if (mx) HIP_TRY(c, launch_lift_mixed(c, w.Y, Uhat, w.Q));   // Q^im_0 = Q(U_n, Uhat_n)
  for (int i = 1; i <= s; ++i) {
    // R^DG(y^ex_i, y^im_{i-1}) (the mixed variables in w.Q belong to y^im_{i-1}; rows of
    // implicit elements in Rdg are never read), y^ex_{i+1}, and the implicit right-hand
    // side rhs = M U_n - dt sum_{j<i} a_ij R^HDG_j: replayed from a graph when enabled
    double coef[4];
    const double* Rs[4];
    for (int j = 0; j < i; ++j) { coef[j] = tab->Ae[4 * i + j]; Rs[j] = Rdg[j]; }
    const double* Rh[3];
    double ch[3];
    for (int j = 0; j < i - 1; ++j) { ch[j] = dt * tab->Ai[3 * (i - 1) + j]; Rh[j] = Rhdg[j]; }
    std::vector<double> key = {dt, (double)i};
    key.insert(key.end(), coef, coef + i);
    key.insert(key.end(), ch, ch + i - 1);
    if (c->mms_on) key.push_back(c->t_now);          // the source depends on the time
    if (tape) HIP_TRY(c, hipMemcpyAsync(tape->Ydg[i - 1], w.Y, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
    const int tdg = c->timer_begin(TM_DG);
    imex_status se = run_captured(c, i - 1, key, [&]() -> imex_status {
      HIP_TRY(c, launch_dg_trace(c, w.Y, mx ? w.Q : nullptr, w.trace));
      HIP_TRY(c, launch_dg_residual(c, w.Y, w.trace, Rdg[i - 1]));
      if (c->mms_on) {
        // the source at the explicit stage time: R^DG_i - b(t_n + cbar_i dt)
        HIP_TRY(c, launch_mms_load(c, c->t_now + ce[i - 1] * dt, c->d_src));
        HIP_TRY(c, launch_rows_axpy(c, 1, 0, -1.0, c->d_src, Rdg[i - 1]));
      }
      HIP_TRY(c, launch_erk_combine(c, w.Un, i, Rs, coef, dt, w.Y));
      if (c->n_im > 0) {
        HIP_TRY(c, launch_mass_rhs(c, w.Un, w.rhs));
        for (int j = 0; j < i - 1; ++j) HIP_TRY(c, launch_rhs_accumulate(c, -ch[j], Rh[j], w.rhs));
      }
      return IMEX_OK;
    });
    c->timer_end(tdg);
    if (se != IMEX_OK) return se;
    if (c->n_im > 0) {
      // Newton initial guess (the converged root does not depend on it): linear
      // extrapolation in stage time from the two previous implicit stage values
      if (i >= 2 && ci[i - 1] - ci[i - 2] > 1e-12 * dt)
        HIP_TRY(c, launch_extrapolate(c, (ci[i] - ci[i - 1]) / (ci[i - 1] - ci[i - 2]), w.Y, w.Yp, Uhat, w.Hp));
      const double dta = dt * tab->Ai[3 * (i - 1) + (i - 1)];
      if (c->mms_on) {
        // the source at the implicit stage time: M y + dt a_ii (R^HDG(y) - b) = rhs
        HIP_TRY(c, launch_mms_load(c, c->t_now + ci[i] * dt, c->d_src));
        HIP_TRY(c, launch_rhs_accumulate(c, dta, c->d_src, w.rhs));
      }
      imex_stats sst{};
      imex_status r = hdg_stage_solve(c, dta, w.rhs, w.Y, Uhat, Rhdg[i - 1], &sst);
      if (r == IMEX_OK && c->mms_on)        // later right-hand sides take R^HDG_i - b_i
        HIP_TRY(c, launch_rows_axpy(c, 2, 0, -1.0, c->d_src, Rhdg[i - 1]));
      if (st) {
        st->newton_its += sst.newton_its;
        st->gmres_its += sst.gmres_its;
        st->newton_last_du = sst.newton_last_du;
        st->t_assemble_ms += sst.t_assemble_ms;
        st->t_solve_ms += sst.t_solve_ms;
        st->n_jacobians += sst.n_jacobians;
        for (int q = 0; q < sst.n_hist && st->n_hist < (int)(sizeof(st->du_hist) / sizeof(double)); ++q)
          st->du_hist[st->n_hist++] = sst.du_hist[q];
      }
      if (r != IMEX_OK) return r;
      if (tape) {
        HIP_TRY(c, hipMemcpyAsync(tape->Ysol[i - 1], w.Y, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
        HIP_TRY(c, hipMemcpyAsync(tape->Hsol[i - 1], Uhat, (size_t)c->n_hf * 4 * c->NP * sizeof(double),
                                  hipMemcpyDeviceToDevice, hs));
      }
    }
  }
  if (!tab->fsal) {
    if (tape) HIP_TRY(c, hipMemcpyAsync(tape->Ydg[s], w.Y, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
    // U^ex_{n+1} = U^ex_n - dt M^-1 sum_j be_j R^DG_j, written over the explicit rows of Y
    double coef[4];
    const double* Rs[4];
    for (int j = 0; j <= s; ++j) { coef[j] = tab->be[j]; Rs[j] = Rdg[j]; }
    std::vector<double> key = {dt, -1.0};
    key.insert(key.end(), coef, coef + s + 1);
    if (c->mms_on) key.push_back(c->t_now);
    const int tdg = c->timer_begin(TM_DG);
    imex_status se = run_captured(c, 4, key, [&]() -> imex_status {
      HIP_TRY(c, launch_dg_trace(c, w.Y, mx ? w.Q : nullptr, w.trace));
      HIP_TRY(c, launch_dg_residual(c, w.Y, w.trace, Rdg[s]));
      if (c->mms_on) {
        HIP_TRY(c, launch_mms_load(c, c->t_now + ce[s] * dt, c->d_src));
        HIP_TRY(c, launch_rows_axpy(c, 1, 0, -1.0, c->d_src, Rdg[s]));
      }
      HIP_TRY(c, launch_erk_combine(c, w.Un, s + 1, Rs, coef, dt, w.Y));
      return IMEX_OK;
    });
    c->timer_end(tdg);
    if (se != IMEX_OK) return se;
  }
  HIP_TRY(c, hipMemcpyAsync(U, w.Y, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  HIP_TRY(c, hipStreamSynchronize(hs));
  c->timers_resolve();
  if (!tape) c->t_now += dt;                 // the clock of the manufactured-solution source
  return IMEX_OK;
}

extern "C" {

imex_status imex_autotune(imex_ctx* c, const double* U, const double* Uhat, int out[4]) {
  if (!c || !U || !out) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (c->n_im > 0 && (c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous) && !Uhat) return fail(c, IMEX_EINVAL, "Uhat required for HDG-MX");
  // explicit residual: elements per workgroup
  if (c->n_ex > 0) {
    float best = 1e30f;
    int pick = 0;
    for (int et : {0, 2, 4, 8, 16, 32}) {
      if (et && !dg_tile_valid(c->K, et)) continue;
      c->dg_tile = et;
      hipEvent_t a, b;
      HIP_TRY(c, hipEventCreate(&a));
      HIP_TRY(c, hipEventCreate(&b));
      imex_status st = dg_residual_async(c, U, Uhat, c->ws.Rstage[7]);
      HIP_TRY(c, hipEventRecord(a, c->stream));
      for (int r = 0; r < 5 && st == IMEX_OK; ++r) st = dg_residual_async(c, U, Uhat, c->ws.Rstage[7]);
      HIP_TRY(c, hipEventRecord(b, c->stream));
      float ms = 1e30f;
      HIP_TRY(c, hipEventSynchronize(b));
      HIP_TRY(c, hipEventElapsedTime(&ms, a, b));
      hipEventDestroy(a);
      hipEventDestroy(b);
      if (st != IMEX_OK) return st;
      if (ms < best) { best = ms; pick = et; }
    }
    c->dg_tile = pick;
  }
  imex_status st = hdg_autotune_gemm(c);
  if (st != IMEX_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timers_resolve();
  for (int t = 0; t < imex_ctx::NTIMER; ++t) { c->tm_ms[t] = 0.0; c->tm_n[t] = 0; }
  c->drop_graphs();
  out[0] = c->dg_tile;
  for (int g = 0; g < 3; ++g) out[1 + g] = c->gemm_tile[g];
  return IMEX_OK;
}

imex_status imex_set_launch_shapes(imex_ctx* c, const int in[4]) {
  if (!c || !in) return fail(c, IMEX_EINVAL, "null argument");
  if (in[0] != 0 && !dg_tile_valid(c->K, in[0])) return fail(c, IMEX_EINVAL, "elements per residual workgroup");
  for (int g = 0; g < 3; ++g) {
    const int t = in[1 + g];
    if (t != 0 && t != 32 && t != 64 && t != 1032 && t != 1064 && !(t >= 2001 && t <= 2011))
      return fail(c, IMEX_EINVAL, "GEMM tile");
  }
  c->dg_tile = in[0];
  for (int g = 0; g < 3; ++g) c->gemm_tile[g] = in[1 + g];
  c->drop_graphs();
  return IMEX_OK;
}

imex_status imex_element_inverse(imex_ctx* c, int set, int* method) {
  if (!c || !method) return fail(c, IMEX_EINVAL, "null argument");
  if (set) {
    if (*method != 0 && *method != 1) return fail(c, IMEX_EINVAL, "element inverse method");
    if (*method == 1 && c->opt.precision != IMEX_FP32_REFINE)
      return fail(c, IMEX_EINVAL, "the matrix-core inverse is the FP32 one");
    c->inv_method = *method;
  }
  *method = c->inv_method;
  return IMEX_OK;
}

imex_status imex_set_graphs(imex_ctx* c, int on) {
  if (!c) return fail(c, IMEX_EINVAL, "null argument");
  if (on && !c->gstream) HIP_TRY(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  c->drop_graphs();
  c->use_graphs = on != 0;
  return IMEX_OK;
}

static bool mx_coupled(const imex_ctx* c) {
  return c->opt.hdg_variant == IMEX_HDG_MX && c->gas.viscous && c->n_im > 0;
}

imex_status imex_vjp_dg_residual(imex_ctx* c, const double* U, const double* Uhat, const double* Rbar, double* Ubar,
                                 double* Uhatbar) {
  if (!c || !U || !Rbar || !Ubar) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (mx_coupled(c) && (!Uhat || !Uhatbar)) return fail(c, IMEX_EINVAL, "HDG-MX coupling needs Uhat and Uhatbar");
  HIP_TRY(c, vjp_alloc(c));
  if (mx_coupled(c))
    HIP_TRY(c, hipMemsetAsync(Uhatbar, 0, sizeof(double) * (size_t)c->n_hf * 4 * c->NP, c->stream));
  HIP_TRY(c, launch_dg_vjp(c, U, Rbar, Ubar, mx_coupled(c) ? Uhat : nullptr, Uhatbar));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return IMEX_OK;
}

// Reverse mode of the explicit ARK step (all elements explicit).  Forward:
// Y_1 = U_n, R_j = R(Y_j), Y_{i+1} = U_n - dt M^-1 sum_{j<=i} Ae[i][j] R_j, and
// U_{n+1} = Y_{s+1} (FSAL) or U_n - dt M^-1 sum_j be_j R_j.  Reverse, stages in
// decreasing order: Rbar_j = -dt M^-1 (be_j Ubar_{n+1} + sum_{i>j} Ae[i-1][j-1] Ybar_i),
// Ybar_j = (dR/dU)^T(Y_j) Rbar_j; Ubar_n = sum_i Ybar_i (+ Ubar_{n+1} if not FSAL).
imex_status imex_vjp_ark_step(imex_ctx* c, const imex_tableau* tab, double dt, const double* U,
                              const double* Ubar_next, double* Ubar) {
  if (!c || !tab || !U || !Ubar_next || !Ubar) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (imex_status ts = check_tableau(c, tab, dt); ts != IMEX_OK) return ts;
  if (c->n_im > 0) return fail(c, IMEX_ENOTIMPL, "step adjoint with an implicit region");
  if (c->mms_on) return fail(c, IMEX_ENOTIMPL, "step adjoint with a manufactured-solution source");
  HIP_TRY(c, vjp_alloc(c));
  Workspace& w = c->ws;
  const int s = tab->s;
  const size_t n = (size_t)c->E * 4 * c->NN;
  hipStream_t hs = c->stream;
  const int nres = tab->fsal ? s : s + 1;           // stages whose residual enters the step
  double** Y = w.vjp_y;                             // Y[0..s]: stage states Y_1..Y_{s+1}
  double** Yb = w.vjp_y + 4;                        // adjoints of Y_1..Y_4 (Y_{s+1} at most)
  double* Rb = w.vjp_y[8];
  double* zero = w.vjp_y[9];
  double* Rs[4] = {w.Rstage[0], w.Rstage[1], w.Rstage[2], w.Rstage[3]};
  HIP_TRY(c, hipMemsetAsync(zero, 0, n * sizeof(double), hs));
  // forward stages
  HIP_TRY(c, hipMemcpyAsync(Y[0], U, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  for (int i = 1; i <= s; ++i) {
    imex_status st = dg_residual_async(c, Y[i - 1], nullptr, Rs[i - 1]);
    if (st != IMEX_OK) return st;
    double coef[4];
    const double* R[4];
    for (int j = 0; j < i; ++j) { coef[j] = tab->Ae[4 * i + j]; R[j] = Rs[j]; }
    HIP_TRY(c, launch_erk_combine(c, U, i, R, coef, dt, Y[i]));
  }
  // reverse
  for (int i = 0; i <= s; ++i) HIP_TRY(c, hipMemsetAsync(Yb[i], 0, n * sizeof(double), hs));
  if (tab->fsal) HIP_TRY(c, hipMemcpyAsync(Yb[s], Ubar_next, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  for (int j = nres; j >= 1; --j) {
    double coef[5];
    const double* T[5];
    int nt = 0;
    if (!tab->fsal) { coef[nt] = tab->be[j - 1]; T[nt++] = Ubar_next; }
    for (int i = j + 1; i <= s + 1; ++i) { coef[nt] = tab->Ae[4 * (i - 1) + (j - 1)]; T[nt++] = Yb[i - 1]; }
    HIP_TRY(c, launch_erk_combine(c, zero, nt, T, coef, dt, Rb));     // Rb = -dt M^-1 sum coef T
    HIP_TRY(c, launch_dg_vjp(c, Y[j - 1], Rb, Yb[j - 1]));
  }
  HIP_TRY(c, hipMemcpyAsync(Ubar, tab->fsal ? zero : Ubar_next, n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  for (int i = 0; i <= s; ++i) HIP_TRY(c, launch_scale_copy(c, Ubar, Ubar, 1.0, Yb[i], 1.0, n));
  HIP_TRY(c, hipStreamSynchronize(hs));
  return IMEX_OK;
}

// Reverse mode of one IMEX step (Alg. imex_scheme_update) with an implicit region.
// The step is recomputed from (U_n, Uhat_n) recording the stage data; then, stages in
// decreasing order, with y^ex_i / y^im_i the explicit / implicit stage values:
//   (d) implicit stage i: transposed condensed solve at the converged stage state,
//       also taking in the adjoint of R^HDG_i from later right-hand sides; gives the
//       adjoint of rhs_i and adds that of the interface data y^ex_{i+1};
//   (c) rhs_i = M U_n - dt sum_{j<i} a_ij R^HDG_j: adjoints of U_n and of R^HDG_j;
//   (b) y^ex_{i+1} = U_n - dt M^-1 sum_{j<=i} ae_{i,j} R^DG_j: adjoints of U_n, R^DG_j;
//   (a) R^DG_i = R^DG(y^ex_i, y^im_{i-1}): residual adjoint into both stage values.
// Uhat_n enters the Newton initial guess and, for HDG-MX, the mixed variables read by
// the first explicit residual; only the latter has an adjoint.
imex_status imex_vjp_imex_step(imex_ctx* c, const imex_tableau* tab, double dt, const double* U, const double* Uhat,
                               const double* Ubar_next, const double* Uhatbar_next, double* Ubar, double* Uhatbar,
                               const double* duinf, double* pbar, imex_stats* st) {
  if (!c || !tab || !U || !Ubar_next || !Ubar) return fail(c, IMEX_EINVAL, "null argument");
  if (!c->regions_set) return fail(c, IMEX_ESTATE, "imex_set_regions first");
  if (imex_status ts = check_tableau(c, tab, dt); ts != IMEX_OK) return ts;
  if (c->mms_on) return fail(c, IMEX_ENOTIMPL, "step adjoint with a manufactured-solution source");
  const bool want_p = duinf && pbar;
  if (want_p) *pbar = 0.0;
  if (c->n_im == 0) {
    if (want_p) return fail(c, IMEX_ENOTIMPL, "far-field parameter adjoint without an implicit region");
    return imex_vjp_ark_step(c, tab, dt, U, Ubar_next, Ubar);
  }
  if (!Uhat) return fail(c, IMEX_EINVAL, "Uhat required with an implicit region");
  const bool mx = mx_coupled(c);
  if (st) std::memset(st, 0, sizeof(*st));
  HIP_TRY(c, vjp_alloc(c));
  Workspace& w = c->ws;
  const int s = tab->s;
  const size_t n = (size_t)c->E * 4 * c->NN, nh = (size_t)c->n_hf * 4 * c->NP;
  hipStream_t hs = c->stream;
  // buffers: tape Ydg[4] Ysol[3] | Uw | yexb[5] yimb[4] Rdgb[5] Rhb[4] rhsb Yb  (state-sized),
  //          Hsol[3] Hw hb[4] (facet-sized)
  constexpr int NSTATE = 4 + 3 + 1 + 5 + 4 + 5 + 4 + 1 + 1, NFAC = 3 + 1 + 4;
  if (w.adj_buf.empty()) {
    for (int i = 0; i < NSTATE + NFAC; ++i) {
      double* p = nullptr;
      HIP_TRY(c, hipMalloc(&p, 8 * (i < NSTATE ? n : std::max<size_t>(nh, 1))));
      w.adj_buf.push_back(p);
    }
    w.bytes += 8 * (NSTATE * n + NFAC * nh);
  }
  double** B = w.adj_buf.data();
  ArkTape tape;
  for (int i = 0; i < 4; ++i) tape.Ydg[i] = B[i];
  for (int i = 0; i < 3; ++i) tape.Ysol[i] = B[4 + i];
  double* Uw = B[7];
  double** yexb = B + 8;       // [i] adjoint of y^ex_i, i = 1..s+1
  double** yimb = B + 13;      // [i] adjoint of y^im_i, i = 0..s
  double** Rdgb = B + 17;      // [j] adjoint of R^DG_j, j = 1..s+1
  double** Rhb = B + 22;       // [j] adjoint of R^HDG_j, j = 1..s
  double* rhsb = B[26];
  double* Yb = B[27];
  for (int i = 0; i < 3; ++i) tape.Hsol[i] = B[NSTATE + i];
  double* Hw = B[NSTATE + 3];
  double** hb = B + NSTATE + 4; // [i] adjoint of Uhat_i, i = 1..s
  // forward recompute with the tape
  HIP_TRY(c, hipMemcpyAsync(Uw, U, n * 8, hipMemcpyDeviceToDevice, hs));
  HIP_TRY(c, hipMemcpyAsync(Hw, Uhat, nh * 8, hipMemcpyDeviceToDevice, hs));
  imex_status fs = ark_step_impl(c, tab, dt, Uw, Hw, nullptr, &tape);
  if (fs != IMEX_OK) return fs;
  for (int i = 8; i < NSTATE; ++i) HIP_TRY(c, hipMemsetAsync(B[i], 0, n * 8, hs));
  for (int i = NSTATE + 4; i < NSTATE + NFAC; ++i) HIP_TRY(c, hipMemsetAsync(B[i], 0, nh * 8, hs));
  HIP_TRY(c, hipMemsetAsync(Ubar, 0, n * 8, hs));
  if (Uhatbar) HIP_TRY(c, hipMemsetAsync(Uhatbar, 0, nh * 8, hs));
  // Far-field parameter: u_inf enters the step only through the residuals' far-field
  // terms, so d(out)/dp along du_inf is the sum over the step's residual evaluations of
  // <their adjoint, dresidual/dp>.  The residual derivatives are exact: the far-field face
  // integrand of R^DG differentiated by a dual number seeded in u_inf, and the derivative
  // A^-(Uhat) du_inf of the far-field facet rows (R^HDG's element rows do not depend on u_inf).
  double pacc = 0.0;
  auto psum = [&](hipError_t launched, double* out) -> imex_status {
    HIP_TRY(c, launched);
    HIP_TRY(c, hipMemcpyAsync(w.hred, w.red, sizeof(double) * 256, hipMemcpyDeviceToHost, hs));
    HIP_TRY(c, hipStreamSynchronize(hs));
    double acc = 0.0;
    for (int b = 0; b < 256; ++b) acc += w.hred[b];
    *out = acc;
    return IMEX_OK;
  };
  // <Rbar, dR^DG/dp> for the explicit residual at Y (the mixed variables of an HDG-MX
  // neighbour do not depend on u_inf)
  auto p_dg = [&](const double* Y, const double*, const double* Rb) -> imex_status {
    if (!want_p) return IMEX_OK;
    double d = 0.0;
    const imex_status r = psum(launch_dg_param_dot(c, duinf, Y, Rb, w.red, 256), &d);
    pacc += d;
    return r;
  };
  // implicit stage at (Y, H) with the solution (lam, lamhat) of its transposed system:
  // -<lamhat, dh/dp> (the element rows' terms <Rhbar, dR^HDG/dp> and <lam, dt_a dR^HDG/dp>
  // vanish)
  auto p_hdg = [&](double, const double*, const double* H, const double*, const double*) -> imex_status {
    if (!want_p) return IMEX_OK;
    double d = 0.0;
    const imex_status r = psum(launch_hdg_param_dot(c, duinf, H, adjoint_facet_solution(c), w.red, 256), &d);
    pacc -= d;
    return r;
  };
  // HDG-MX: the explicit residual of stage i reads the mixed variables lifted from
  // (y^im_{i-1}, Uhat_{i-1}); their adjoint goes to that facet state as well
  auto hin = [&](int i) -> const double* { return i >= 2 ? tape.Hsol[i - 2] : Uhat; };
  auto hout = [&](int i) -> double* { return i >= 2 ? hb[i - 1] : (Uhatbar ? Uhatbar : Hw); };
  // the step's outputs: U_{n+1} = (y^ex_{s+1} | final update, y^im_s), Uhat_{n+1} = Uhat_s
  HIP_TRY(c, launch_rows_axpy(c, 2, 0, 1.0, Ubar_next, yimb[s]));
  if (Uhatbar_next) HIP_TRY(c, launch_scale_copy(c, hb[s], hb[s], 1.0, Uhatbar_next, 1.0, nh));
  if (tab->fsal) {
    HIP_TRY(c, launch_rows_axpy(c, 1, 0, 1.0, Ubar_next, yexb[s + 1]));
  } else {
    HIP_TRY(c, launch_rows_axpy(c, 1, 0, 1.0, Ubar_next, Ubar));
    for (int j = 1; j <= s + 1; ++j) HIP_TRY(c, launch_rows_axpy(c, 1, 2, -dt * tab->be[j - 1], Ubar_next, Rdgb[j]));
    HIP_TRY(c, launch_dg_vjp(c, tape.Ydg[s], Rdgb[s + 1], Yb, mx ? tape.Hsol[s - 1] : nullptr, hb[s]));
    if (imex_status r = p_dg(tape.Ydg[s], tape.Hsol[s - 1], Rdgb[s + 1]); r != IMEX_OK) return r;
    HIP_TRY(c, launch_rows_axpy(c, 1, 0, 1.0, Yb, yexb[s + 1]));
    HIP_TRY(c, launch_rows_axpy(c, 2, 0, 1.0, Yb, yimb[s]));
  }
  int gm_total = 0;
  for (int i = s; i >= 1; --i) {
    // (d) implicit stage i
    HIP_TRY(c, hipMemsetAsync(rhsb, 0, n * 8, hs));
    int its = 0;
    const double dta = dt * tab->Ai[3 * (i - 1) + (i - 1)];
    imex_status r = hdg_stage_adjoint(c, dta, tape.Ysol[i - 1], tape.Hsol[i - 1], Rhb[i], yimb[i], hb[i], rhsb,
                                      yexb[i + 1], &its);
    if (r != IMEX_OK) return r;
    if ((r = p_hdg(dta, tape.Ysol[i - 1], tape.Hsol[i - 1], Rhb[i], rhsb)) != IMEX_OK) return r;
    gm_total += its;
    // (c) right-hand side
    HIP_TRY(c, launch_rows_axpy(c, 2, 1, 1.0, rhsb, Ubar));
    for (int j = 1; j < i; ++j) HIP_TRY(c, launch_rows_axpy(c, 2, 3, -dt * tab->Ai[3 * (i - 1) + (j - 1)], rhsb, Rhb[j]));
    // (b) explicit stage value y^ex_{i+1}
    HIP_TRY(c, launch_rows_axpy(c, 1, 0, 1.0, yexb[i + 1], Ubar));
    for (int j = 1; j <= i; ++j) HIP_TRY(c, launch_rows_axpy(c, 1, 2, -dt * tab->Ae[4 * i + (j - 1)], yexb[i + 1], Rdgb[j]));
    // (a) explicit residual of stage i at (y^ex_i, y^im_{i-1})
    HIP_TRY(c, launch_dg_vjp(c, tape.Ydg[i - 1], Rdgb[i], Yb, mx ? hin(i) : nullptr, hout(i)));
    if ((r = p_dg(tape.Ydg[i - 1], hin(i), Rdgb[i])) != IMEX_OK) return r;
    HIP_TRY(c, launch_rows_axpy(c, 1, 0, 1.0, Yb, i >= 2 ? yexb[i] : Ubar));
    HIP_TRY(c, launch_rows_axpy(c, 2, 0, 1.0, Yb, yimb[i - 1]));
  }
  HIP_TRY(c, launch_rows_axpy(c, 2, 0, 1.0, yimb[0], Ubar));
  HIP_TRY(c, hipStreamSynchronize(hs));
  c->timers_resolve();
  if (st) st->gmres_its = gm_total;
  if (want_p) *pbar = pacc;
  return IMEX_OK;
}

static_assert(imex_ctx::NTIMER == IMEX_NTIMERS, "timer count of the C ABI");

imex_status imex_kernel_times(imex_ctx* c, double out[2 * IMEX_NTIMERS], int reset) {
  if (!c || !out) return fail(c, IMEX_EINVAL, "null argument");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timers_resolve();
  for (int t = 0; t < imex_ctx::NTIMER; ++t) {
    out[2 * t] = c->tm_ms[t];
    out[2 * t + 1] = (double)c->tm_n[t];
    if (reset) { c->tm_ms[t] = 0.0; c->tm_n[t] = 0; }
  }
  return IMEX_OK;
}

imex_status imex_set_timer_mask(imex_ctx* c, unsigned mask) {
  if (!c) return fail(c, IMEX_EINVAL, "null argument");
  if (mask >> IMEX_NTIMERS) return fail(c, IMEX_EINVAL, "timer mask has bits beyond the phases");
  c->timer_mask = mask;
  return IMEX_OK;
}

imex_status imex_conservation_sums(imex_ctx* c, const double* U, double out[4]) {
  if (!c || !U || !out) return fail(c, IMEX_EINVAL, "null argument");
  int nb = 0;
  HIP_TRY(c, launch_mass_sums(c, U, c->ws.Rstage[7], &nb));
  std::vector<double> part((size_t)nb * 4);
  HIP_TRY(c, hipMemcpyAsync(part.data(), c->ws.Rstage[7], part.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * 4 + v];
    out[v] = s;
  }
  return IMEX_OK;
}

void imex_destroy(imex_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  c->timers_resolve();
  for (hipEvent_t e : c->ev_free) hipEventDestroy(e);
  c->ev_free.clear();
  for (hipEvent_t e : {c->pev_f[0], c->pev_f[1], c->pev_g[0][0], c->pev_g[0][1], c->pev_g[1][0], c->pev_g[1][1]})
    if (e) hipEventDestroy(e);
  c->drop_graphs();
  if (c->gstream) hipStreamDestroy(c->gstream);
  c->gstream = nullptr;
  free_regions(c);
  Workspace& w = c->ws;
  for (double** p : {&w.trace, &w.Q, &w.Un, &w.Y, &w.rhs, &w.Yp}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  for (int r = 0; r < 8; ++r) {
    if (w.Rstage[r]) hipFree(w.Rstage[r]);
    w.Rstage[r] = nullptr;
  }
  for (double** p : {&w.vjp_tu, &w.vjp_tr, &w.vjp_pf, &w.vjp_pv, &w.vjp_tq, &w.vjp_pq, &w.vjp_qb, &w.vjp_q,
                     &w.vjp_hb}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  for (int r = 0; r < 10; ++r) {
    if (w.vjp_y[r]) hipFree(w.vjp_y[r]);
    w.vjp_y[r] = nullptr;
  }
  for (double** p : {&c->d_hx, &c->d_hy, &c->d_dts, &c->d_xy0, &c->d_src}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  for (int** p : {&c->d_nbr, &c->d_bcf}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  if (c->d_imp) hipFree(c->d_imp);
  if (c->d_tab) hipFree(c->d_tab);
  delete c;
}

}  // extern "C"
