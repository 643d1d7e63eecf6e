// Internal state of an imex_ctx and the launch interfaces of the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/imexhdg.h"
#include "device_common.h"

namespace imex {

// HDG facet kinds as seen from an implicit element's face
enum FaceKind { FK_INTERIOR = 0, FK_INTERFACE = 1, FK_FARFIELD = 2, FK_WALL = 3 };

struct DeviceMesh {
  int E, K;
  const double* hx;         // [E]
  const double* hy;         // [E]
  const int* nbr;           // [E][4] neighbour element or -1
  const int* bcf;           // [E][4] boundary type where nbr == -1
  const unsigned char* imp; // [E]
  const BasisTable* tab;
  const double* dts;        // [E] time-step scale of each element's instance, or null (all 1)
};

// one structured mesh of a (possibly multi-instance) context; elements e_off ..
// e_off + nx ny - 1, element e_off + i + nx j covers [xg_i, xg_i+1] x [yg_j, yg_j+1]
struct Inst {
  int nx = 0, ny = 0, e_off = 0;
  int bc[4] = {0, 0, 0, 0};
  double dt_scale = 1.0;
  std::vector<double> xg, yg;
};

// per-element time-step factor (1 without a scale table)
__device__ __forceinline__ double elem_dt(const DeviceMesh& m, int e) { return m.dts ? m.dts[e] : 1.0; }

// Implicit-region tables (device)
struct DeviceHDG {
  int n_im, n_hf;
  const int* im_list;       // [n_im] element ids
  const int* face_kind;     // [n_im][4]
  const int* efacet;        // [n_im][4] HDG facet index of each face
  const int* hf_side;       // [n_hf][2] implicit-list position of the (lower, upper) side or -1
  const int* hf_face;       // [n_hf][2] local face of that side
  const int* hf_elem;       // [n_hf][2] element id of each side or -1
  // two-column Schwarz windows of the facet preconditioner
  int n_win;
  const int* win_off;       // [n_win+1] offsets (in super-rows) of each window
  const int* win_slot;      // [n_superrows][5] HDG facet of each slot or -1
  const int* win_own;       // [n_superrows][5] 1 if the window writes that facet's result
  int n_sr;
  const int* sr_flags;      // [n_superrows] bit 0: has a predecessor, bit 1: has a successor
};

struct Workspace {
  double* trace = nullptr;      // [E][4][NQ][8] face traces: U and F^nu . n
  double* Q = nullptr;          // [E][5][NN] mixed variables of implicit elements (HDG-MX)
  double* Rstage[8] = {};       // ARK stage residuals, [E][4][NN] each
  double* Un = nullptr;         // copy of U at t_n
  double* Y = nullptr;          // stage state
  double* rhs = nullptr;        // implicit stage right-hand side
  double* Yp = nullptr;         // previous implicit stage value (stage predictor)
  double* Hp = nullptr;         // previous facet stage value (stage predictor)
  // implicit Newton.  The linear-algebra buffers hold doubles (IMEX_FP64) or
  // floats (IMEX_FP32_REFINE); the Newton residual column of blk is stored in
  // the same type, the state, residual evaluation and Krylov vectors stay FP64.
  void* blk = nullptr;          // per implicit element: augmented system [[K C f],[D E h]] (becomes [[. . .],[D S h-DK^-1f]])
  void* scr = nullptr;          // per implicit element: HDG-MX mixed blocks [A12; A32] and M_Q^-1 [A21 A23]
  double* rec = nullptr;        // per implicit element: HDG-MX point-wise Jacobians (assembly -> contraction)
  double* hres = nullptr;       // per implicit element: its share of the facet residuals h (FP64) [NF]
  void* Kinv = nullptr;         // per implicit element: K^-1 [NU][NU]
  void* X = nullptr;            // per implicit element: K^-1 [C f]  [NU][NF+1]
  void* Wd = nullptr;           // per window super-row: inverse of the eliminated diagonal block
  void* Wg = nullptr;           // per window super-row: B_r D_{r-1}^-1 (facet rows x previous super-row)
  void* Wc = nullptr;           // per window super-row: D_r^-1 C_r, coupling to the next super-row
  double* Wy = nullptr;         // per window super-row: sweep vectors y_r, w_r (NB each) and z_r on H (NH)
  double* gH = nullptr;         // GMRES Hessenberg, rotations, g, residual history, scalars (device)
  double* gm = nullptr;         // GMRES basis and vectors
  // vector-Jacobian products (allocated on first use)
  double* vjp_tu = nullptr;     // [E][4][NQ][12] face traces of U (value, d/dxi, d/deta)
  double* vjp_tr = nullptr;     // [E][4][NQ][12] face traces of the residual adjoint
  double* vjp_pf = nullptr;     // [E][4][NQ][12] face-point adjoints (trace, physical gradient)
  double* vjp_pv = nullptr;     // [E][NQV][12] volume-point adjoints
  double* vjp_y[10] = {};       // stage states, their adjoints and scratch ([E][4][NN] each)
  double* vjp_tq = nullptr;     // [E][4][NQ][5] face traces of the mixed variables (HDG-MX)
  double* vjp_pq = nullptr;     // [E][4][NQ][5] their adjoints
  double* vjp_qb = nullptr;     // [E][5][NN] adjoint of the mixed variables
  double* vjp_q = nullptr;      // [E][5][NN] lifted mixed variables
  double* vjp_hb = nullptr;     // [n_im][4][4][NP] element shares of the facet adjoint
  double* adj_P = nullptr;      // [n_hf][NFF][NFF] facet block-Jacobi factors of S^T
  double* adj_w = nullptr;      // [E][4][NN] element scratch of the transposed solve
  std::vector<double*> adj_buf; // step-adjoint tape and adjoints ([E][4][NN] or facet-sized)
  double* adj_rp = nullptr;     // [E][4][NN] residuals at u_inf +- eps du_inf (parameter adjoint)
  double* adj_rm = nullptr;
  double* adj_hp = nullptr;     // [n_im][NF] facet residual shares at u_inf +- eps du_inf
  double* adj_hm = nullptr;
  double* red = nullptr;        // reduction scratch
  double* hred = nullptr;       // pinned host reduction buffer
  double* hgm = nullptr;        // coherent pinned host buffer the GMRES kernels write their residual
                                // estimates into ([0, GM_MAXM] and beta at GM_MAXM + 1), host address
  double* hgm_dev = nullptr;    // the same buffer's device address
  size_t bytes = 0;
};

}  // namespace imex

struct imex_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int E = 0, K = 0, NP = 0, NQ = 0, NN = 0;
  std::vector<imex::Inst> inst;     // the structured meshes (one, or a batch of disjoint ones)
  imex::Gas gas{};
  imex_options opt{};
  imex::BasisTable tab{};
  // host tables
  std::vector<int> nbr, bcf;
  std::vector<unsigned char> imp;
  std::vector<int> im_list, ex_list, face_kind, efacet, hf_side, hf_face, hf_elem;
  std::vector<int> win_off, win_slot, win_own, sr_flags;
  int n_win = 0, n_superrows = 0;
  int n_im = 0, n_ex = 0, n_hf = 0;
  bool dg_farfield = false;     // some explicit element has a far-field boundary face
  // manufactured-solution source (imex_set_mms_source): wave numbers, frequency, clock
  bool mms_on = false;
  double mms[3] = {0.0, 0.0, 0.0};
  double t_now = 0.0;
  double* d_xy0 = nullptr;      // [E][2] lower-left corner of each element
  double* d_src = nullptr;      // [E][4][NN] source load of one stage time
  bool regions_set = false;
  // launch shapes (0 = built-in default), chosen by imex_autotune
  int dg_tile = 0;              // explicit elements per workgroup of the residual kernel
  int gemm_tile[3] = {0, 0, 0}; // output tile (64 or 32) of the elimination, K^-1 [C f] and Schur GEMMs
  int inv_method = 0;           // K^-1: 0 register Gauss-Jordan, 1 blocked Gauss-Jordan on MFMA (FP32)
  // facet preconditioner reuse across Newton iterations, stages and steps
  bool prec_valid = false;      // factors match a recent system
  bool prec_fresh = false;      // the next GMRES solve is the first after a refactorisation
  int prec_base = 0;            // GMRES iterations of that first solve
  int prec_extra = 0;           // GMRES iterations above prec_base since then
  double newton_q2 = 0.0;       // contraction of the second Newton correction in the last stage (0: none yet)
  double prec_dt_a = 0.0;       // dt a_ii of the factorised system
  // refactorisation cost in GMRES iterations, from the device time of the last
  // factorisation over that of an iteration (events read once the stream has passed them)
  double prec_cost_its = 8.0;
  double prec_fac_ms = 0.0, prec_it_ms = 0.0;
  hipEvent_t pev_f[2] = {nullptr, nullptr};                  // factorisation begin, end
  hipEvent_t pev_g[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // GMRES begin, end (two slots)
  bool pev_fset = false, pev_gset[2] = {false, false};
  int pev_gits[2] = {0, 0}, pev_slot = 0;
  // device copies
  double *d_hx = nullptr, *d_hy = nullptr, *d_dts = nullptr;
  int *d_nbr = nullptr, *d_bcf = nullptr;
  unsigned char* d_imp = nullptr;
  imex::BasisTable* d_tab = nullptr;
  int *d_im_list = nullptr, *d_ex_list = nullptr, *d_face_kind = nullptr, *d_efacet = nullptr;
  int *d_hf_side = nullptr, *d_hf_face = nullptr, *d_hf_elem = nullptr;
  int *d_win_off = nullptr, *d_win_slot = nullptr, *d_win_own = nullptr, *d_sr_flags = nullptr;
  std::vector<int> ex_ifacet;           // [E][4] interface HDG facet across each face of explicit elements, or -1
  int* d_ex_ifacet = nullptr;
  bool adj_mode = false;                // GMRES solves S^T (reverse mode)
  imex::Workspace ws;
  std::string err;
  // hipGraph replay of each stage's explicit sequence (imex_set_graphs)
  struct StageGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<double> key;
  };
  bool use_graphs = false;
  bool capturing = false;
  hipStream_t gstream = nullptr;
  StageGraph sg[5];
  std::map<int, hipGraphExec_t> gm_graphs;   // GMRES inner blocks by (first column, length, adjoint mode)
  int gm_hist[8] = {};                       // iterations of the last GMRES solve of each kind
  void drop_graphs();
  // device-time accounting per phase (hipEvents resolved at synchronisation points)
  static constexpr int NTIMER = 11;
  double tm_ms[NTIMER] = {};
  long long tm_n[NTIMER] = {};
  std::vector<hipEvent_t> ev_free;
  struct Pending { int tag; hipEvent_t a, b; };
  std::vector<Pending> ev_pending;
  unsigned timer_mask = ~0u;          // bit t: phase t records its hipEvents
  int timer_begin(int tag);
  void timer_end(int idx);
  void timers_resolve();
  imex::DeviceMesh dmesh() const {
    return imex::DeviceMesh{E, K, d_hx, d_hy, d_nbr, d_bcf, d_imp, d_tab, d_dts};
  }
  imex::DeviceHDG dhdg() const {
    return imex::DeviceHDG{n_im,      n_hf,  d_im_list, d_face_kind, d_efacet,    d_hf_side, d_hf_face,
                           d_hf_elem, n_win, d_win_off, d_win_slot, d_win_own, n_superrows, d_sr_flags};
  }
};

// timer tags
namespace imex {
enum TimerTag { TM_DG = 0, TM_ASSEMBLE = 1, TM_ELIMINATE = 2, TM_CONDENSE = 3, TM_FACET = 4, TM_GMRES = 5,
                TM_BACKSUB = 6, TM_PRECOND = 7, TM_POINTS = 8, TM_CONTRACT = 9, TM_INVERT = 10 };
}

// kernel launchers (dg.hip)
namespace imex {
// static device scratch of imex_dg_residual_noalloc: 96 MiB per device
constexpr size_t STATIC_SCRATCH_DOUBLES = (size_t)96 << 17;
constexpr int MAX_DEVICES = 64;
hipError_t static_scratch_init(int device);   // resolve the device address (device current)
double* static_scratch(int device);           // that address, or null before a successful init
hipError_t launch_fill_zero(const imex_ctx* c, double* x, size_t n);
// b[e][v][n] = int_T S_v(x, t) phi_n of the manufactured-solution source at time t
hipError_t launch_mms_load(const imex_ctx* c, double t, double* b);
hipError_t launch_dg_trace(const imex_ctx* c, const double* U, const double* Q, double* trace);
hipError_t launch_dg_residual(const imex_ctx* c, const double* U, const double* trace, double* R);
hipError_t launch_erk_combine(const imex_ctx* c, const double* Un, int nterms, const double* const* R,
                              const double* coef, double dt, double* Y);
hipError_t launch_mass_sums(const imex_ctx* c, const double* U, double* partial, int* nblocks);
hipError_t launch_scale_copy(const imex_ctx* c, const double* src, double* dst, double a, const double* add,
                             double b, size_t n);
bool dg_tile_valid(int K, int et);
// hdg.hip
hipError_t launch_init_facets(const imex_ctx* c, const double* U, double* Uhat);
hipError_t launch_init_facets_vjp(const imex_ctx* c, const double* Hb, double* Ub);
hipError_t launch_wall_shear(const imex_ctx* c, const double* Q, double* part);
hipError_t launch_hdg_residual(imex_ctx* c, double dt_a, const double* Y, const double* H, double* Rh);
const double* adjoint_facet_solution(const imex_ctx* c);
hipError_t launch_param_dot(const imex_ctx* c, int kind, int scaled, const double* a, const double* b, double* part,
                            int nblk);
// exact <Rbar, dR^DG/dp> and <lamhat, dh/dp> along u_inf + p du (per-block partial sums)
hipError_t launch_dg_param_dot(const imex_ctx* c, const double* du, const double* U, const double* Rb, double* part,
                               int nblk);
hipError_t launch_hdg_param_dot(const imex_ctx* c, const double* du, const double* H, const double* lam, double* part,
                                int nblk);
hipError_t launch_wall_shear_qbar(const imex_ctx* c, double scale, double* Qb);
hipError_t launch_lift_mixed(const imex_ctx* c, const double* U, const double* Uhat, double* Q);
hipError_t launch_mass_rhs(const imex_ctx* c, const double* Un, double* rhs);
hipError_t launch_rhs_accumulate(const imex_ctx* c, double b, const double* R, double* rhs);
hipError_t launch_extrapolate(const imex_ctx* c, double coef, double* Y, double* Yp, double* Uhat, double* Hp);
imex_status hdg_stage_solve(imex_ctx* c, double dt_a, const double* rhs, double* U, double* Uhat, double* R_out,
                            imex_stats* st);
imex_status hdg_local_system(imex_ctx* c, double dt_a, const double* rhs, const double* U, const double* Uhat,
                             double* f, double* h, double* K, double* C, double* D, double* E);
size_t hdg_workspace_bytes(const imex_ctx* c);
imex_status hdg_autotune_gemm(imex_ctx* c);
imex_status hdg_stage_adjoint(imex_ctx* c, double dt_a, const double* Y, const double* H, const double* Rhbar,
                              double* ybar, double* hbar, double* rhsbar, double* yexbar, int* gmres_its);
hipError_t launch_rows_axpy(const imex_ctx* c, int rows, int fac, double a, const double* in, double* out);
hipError_t launch_lift_vjp(const imex_ctx* c, const double* U, const double* Uhat, const double* Qb, double* Ub,
                           double* Hb, double* Uhatbar);
// vjp.hip
hipError_t vjp_alloc(imex_ctx* c);
hipError_t launch_dg_vjp(imex_ctx* c, const double* U, const double* Rb, double* Ub, const double* Uhat = nullptr,
                         double* Uhatbar = nullptr);
imex_status hdg_alloc(imex_ctx* c);
}  // namespace imex
