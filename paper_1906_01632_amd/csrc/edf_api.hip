// C-ABI of the Elder-flow solver: problem set-up, the Newton / BiCGStab / V-cycle
// drivers, state I/O and statistics.  Every numerical step runs in the kernels of
// fv_kernels.hip, mg_kernels.hip and krylov_kernels.hip; this file only sizes
// buffers, enqueues kernels on the caller's stream and makes the per-sample
// decisions (convergence, line search) that need host control.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "adjoint.h"
#include "gpc.h"
#include "edf.h"
#include "edf_internal.h"

using namespace edf;

namespace {

struct Level {
  Geom g;
  Phys ph;
  size_t cells = 0;
  double* phi = nullptr;  // [S][cells]
  double* K = nullptr;
  double* u = nullptr;    // state on this level [S][N][2] (level 0: the Newton iterate)
  double* A64 = nullptr;  // [S][Np x 108] colour-major, packed (level 0: exact Jacobian)
  double* AV64 = nullptr; // level 0 in FP64 mode: the V-cycle matrix
  float* A32 = nullptr;   // V-cycle matrix in mixed mode
  _Float16* A16 = nullptr;  // finest level with EDF_PREC_MIXED_F16: D^{-1} A in FP16 (Dinv
                            // then holds the diagonal blocks D themselves, FP32)
  void* Dinv = nullptr;   // [S][Np x 4], V-cycle precision
  void* LF = nullptr;     // vertical-line smoother: [S][Np x 8] column block-LU factors
  void* x = nullptr;      // V-cycle vectors [S][Np][2] colour-major, V-cycle precision
  void* b = nullptr;
  void* r = nullptr;
  // the group's first sample in the allocations this level shares with the levels of
  // other groups on the same grid (V-cycle arrays; see plan_pools)
  int slot = 0;
  int line_cols = 16;  // tile shape of the line sweep: columns per workgroup (autotuned)
};

// one timed launch (edf_profile)
struct ProfRec {
  int pair, kind;  // kind 0: one smoother launch, 1: one whole V-cycle
  double bytes;    // algorithmic bytes
  bool large;      // a smoother launch of more than kLargeLaunch bytes
};
// launches that move more than this are beyond the 256 MiB last-level cache, so their
// bandwidth is HBM bandwidth; smaller ones may partly hit the cache
constexpr double kLargeLaunch = 256.0 * 1024 * 1024;

struct Group {
  edf_group_desc d{};
  std::vector<int> slots;  // Level::slot of every level, planned before allocation
  long list_ver = 0;       // bumped whenever the V-cycle sample list changes
  bool in_krylov = false;  // inside BiCGStab (merged V-cycles, concurrent_groups = 2)
  // groups step concurrently, each from its own host thread on its own stream
  hipStream_t st = nullptr;
  int* h_int = nullptr;  // pinned host staging [S]
  // the samples the V-cycle launches run over (device list, pinned host copy, count)
  int* d_list = nullptr;
  int* h_list = nullptr;
  int n_list = 0;
  double* h_dbl = nullptr;
  KrylovScalars* h_ks = nullptr;
  // smoother and V-cycle timing: event pairs around every timed launch
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<ProfRec> prof_pending;
  // [0] timed smoother launches, [1] V-cycles, [2] the timed smoother launches whose
  // algorithmic bytes exceed kLargeLaunch (working sets beyond the last-level cache)
  double prof_count[4] = {0, 0, 0, 0}, prof_ms[4] = {0, 0, 0, 0}, prof_bytes[4] = {0, 0, 0, 0};
  // every smoother launch, timed or not: all of them, and those beyond kLargeLaunch
  double prof_all_count[2] = {0, 0}, prof_all_bytes[2] = {0, 0};
  long long prof_tick = 0;
  int S = 0, s0 = 0, L = 0;
  std::vector<Level> lv;
  size_t N = 0, n = 0;  // finest vertices, unknowns
  double *u = nullptr, *u_old = nullptr, *F = nullptr, *Ft = nullptr, *ut = nullptr;
  double *kx = nullptr, *kr = nullptr, *krh = nullptr, *kp = nullptr, *kv = nullptr,
         *ks_ = nullptr, *kt = nullptr, *kph = nullptr, *ksh = nullptr;
  KrylovScalars* ks = nullptr;
  double* part = nullptr;
  int *nmask = nullptr, *active = nullptr, *lsmask = nullptr;
  double *norms = nullptr, *lam = nullptr, *dts = nullptr, *crange = nullptr, *eta = nullptr;
  double* u0 = nullptr;  // state at the start of the current step (restart point)
  // opts.predictor: the state at the start of the previous step, and that step's length
  // per sample when it was one implicit-Euler step (0: no usable history)
  double* u_prev = nullptr;
  std::vector<double> pred_dt;
  double* Minv = nullptr;
  int *piv = nullptr, *gj_status = nullptr;
  int n_coarse = 0;
  int n_active = 0;  // samples active in the current Krylov chunk (known at chunk start)
  int fuse_from = -1;  // levels from here on run in the fused launch (-1: not chosen yet)
  int min_fuse = 0;    // 1 when the finest level has an FP16 matrix (separate launches)
  void* fdesc = nullptr;  // device copy of the fused-bottom description (FusedLevels<T>)
  int fdesc_l0 = -1;      // the first fused level it describes (-1: not written yet)
  // captured V-cycles (graph_vcycle): one executable graph per launch configuration
  struct VGraph {
    int l0, n_list, listed, zs;
    const double* in;
    double* out;
    const int* mask;
    hipGraphExec_t exec;
  };
  std::vector<VGraph> vgraphs;
  // the matrices are the adjoint's transposed ones: their V-cycle keeps the general
  // residual b - A x after the zero-start sweep
  bool transposed = false;
  std::vector<double> tune_ms;  // V-cycle time per candidate fuse_from (autotuning)
  // per sample: halvings to start the next step with, steps since the last retry,
  // steps to wait before trying one halving less, whether this step is such a try
  // (opts.substep_memory)
  std::vector<int> h_start, clean, wait, probing;
  // per sample: the failure status of the step that failed (EDF_SAMPLE_OK: none); a
  // failed sample is not advanced again until edf_set_state resets it
  std::vector<int> fail_status;
  // FP64 mass balance of the current step: accumulators [S][8] and block partials
  double* bal = nullptr;
  double* bal_part = nullptr;
  // trajectory recorded by edf_solve for edf_adjoint (allocated on first use)
  double* ckpt = nullptr;      // [S][ckpt_cap][n]: states at steps 0, k, 2k, ... and the last
  size_t ckpt_cap = 0;
  double* seg = nullptr;       // [S][seg_cap][n]: the states of one segment of k steps
  size_t seg_cap = 0;
  std::vector<std::vector<int>> H;  // [step][S]: halvings of every recorded step
  std::vector<int> traj_fail;       // [S]: the sample failed during the recorded steps
  double* sub = nullptr;       // [S][sub_cap][n]: the sub-step states of one step
  size_t sub_cap = 0;
  double* lam_next = nullptr;  // [S][n]
  double* tmpA = nullptr;      // [S][108][Np_0] FP64 scratch for transposition
  int* idx = nullptr;          // [S]
  double* g4 = nullptr;        // [S][4]
  std::vector<edf_step_stats> stats;
};

// a group's request for one V-cycle, out = M^{-1} in (merged V-cycles)
struct MergeReq {
  Group* G;
  const double* in;
  double* out;
  const int* mask;
  bool done = false;
};

// arrays of a V-cycle level that live in the shared allocations of its grid
enum PoolKind { kPoolVA64, kPoolA32, kPoolDinv, kPoolLF, kPoolR, kPoolB, kPoolX, kPoolMinv };

}  // namespace

struct edf_problem {
  edf_physics phys{};
  edf_solver_opts opts{};
  hipStream_t st = nullptr;
  std::vector<Group> groups;
  int S_total = 0;
  bool params_set = false;
  std::string err;
  std::mutex mu;  // guards err and allocs (groups run on several host threads)
  int device = 0;  // the device current at creation; every group thread uses it
  std::vector<void*> allocs;
  double* dxi = nullptr;  // parameters on the device [S_total][max(n_xi, 1)]
  // polynomial chaos surrogate of the last edf_gpc_project (device, grow-only)
  int gpc_nc = 0, gpc_M = 0, gpc_deg = 0, gpc_trunc = 0, gpc_Nc = 0;
  double* gpc_buf = nullptr;  // C [nc][Nc], Q [nc], W [nc][S], w [S], F [S][Nc], mean/var
  size_t gpc_cap = 0;
  int* gpc_ibuf = nullptr;    // idx [nc][M], then exceedance counts
  size_t gpc_icap = 0;
  double* gpc_pts = nullptr;  // exceedance points [Ns][M], then probabilities [Nc]
  size_t gpc_pcap = 0;
  // the trajectory of the last edf_solve with checkpoint_every > 0, valid until a step,
  // a new state or new parameters change it
  bool traj_valid = false;
  bool recording = false;  // edf_solve is recording a trajectory (no extrapolated starts)
  int traj_k = 0, traj_n = 0;
  double traj_dt = 0.0;
  // staging for edf_set_parameters: the new parameters are checked before they replace
  // the current ones
  double* dxi_new = nullptr;
  int* bad = nullptr;  // [S_total] flags of the check
  // V-cycle arrays of levels on equal grids share one allocation per array kind, the
  // groups' samples side by side (slots), so that one launch can serve several groups
  struct Pool {
    int nx, ny, nz, kind;
    size_t per_sample;
    char* base;
  };
  std::vector<Pool> pools;
  std::map<std::tuple<int, int, int>, int> pool_slots;  // slots per grid
  // merged V-cycles (concurrent_groups = 2): the groups' host threads meet before each
  // V-cycle; when every group inside BiCGStab has arrived, one of them launches the
  // V-cycles of all, one launch per shared grid level
  std::mutex mg_mu;
  std::condition_variable mg_cv;
  int mg_in = 0;                       // groups inside BiCGStab
  std::vector<MergeReq*> mg_wait;
  struct ListBuf {
    std::vector<long> key;   // the (group, level) pairs it serves
    std::vector<long> vkey;  // their list versions and counts when it was built
    int* d = nullptr;
    int n = 0;
  };
  std::vector<ListBuf> mg_lists;
  struct BottomDesc {
    std::vector<long> key;
    void* d = nullptr;
  };
  std::vector<BottomDesc> mg_bottoms;
  // statistics buffers (allocated on first use)
  double* mom_f = nullptr;
  double* mom_w = nullptr;
  double* mom_out = nullptr;
  size_t mom_cap = 0;
};

namespace {

void set_err(edf_problem* pb, const std::string& msg) {
  if (!pb) return;
  std::lock_guard<std::mutex> lock(pb->mu);
  pb->err = msg;
}

#define EDF_TRY(expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      set_err(pb, std::string(#expr ": ") + hipGetErrorString(e_));     \
      return EDF_ERR_HIP;                                               \
    }                                                                   \
  } while (0)

#define EDF_CHECK_LAUNCH()                                                   \
  do {                                                                       \
    hipError_t e_ = hipGetLastError();                                       \
    if (e_ != hipSuccess) {                                                  \
      set_err(pb, std::string("kernel launch: ") + hipGetErrorString(e_));   \
      return EDF_ERR_HIP;                                                    \
    }                                                                        \
  } while (0)

edf_status fail(edf_problem* pb, edf_status code, const std::string& msg) {
  set_err(pb, msg);
  return code;
}

template <typename T>
edf_status dalloc(edf_problem* pb, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return EDF_OK;
  void* q = nullptr;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(pb, EDF_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) +
                                     " bytes failed");
  }
  {
    std::lock_guard<std::mutex> lock(pb->mu);
    pb->allocs.push_back(q);
  }
  *p = static_cast<T*>(q);
  return EDF_OK;
}

Geom make_geom(int nx, int ny, int nz, const edf_physics& P) {
  Geom g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.N = nx * ny * nz;
  g.hx = P.lx / (nx - 1);
  g.hy = P.ly / (ny - 1);
  g.hz = P.lz / (nz - 1);
  int off = 0;
  for (int col = 0; col < 8; ++col) {
    const int ci = col & 1, cj = (col >> 1) & 1, ck = col >> 2;
    const int mx = (nx - ci + 1) / 2, my = (ny - cj + 1) / 2, mz = (nz - ck + 1) / 2;
    g.mx[col] = mx;
    g.my[col] = my;
    g.cnt[col] = mx * my * mz;
    g.off[col] = off;
    off += ceil_div(g.cnt[col], kTile) * kTile;
  }
  g.off[8] = off;
  const double tol = 1e-9 * std::max(P.lx, P.ly);
  g.pi0 = std::max(0, (int)std::ceil((P.patch[0] - tol) / g.hx));
  g.pi1 = std::min(nx - 1, (int)std::floor((P.patch[1] + tol) / g.hx));
  g.pj0 = std::max(0, (int)std::ceil((P.patch[2] - tol) / g.hy));
  g.pj1 = std::min(ny - 1, (int)std::floor((P.patch[3] + tol) / g.hy));
  if (g.pj0 > g.pj1) g.pi0 = g.pi1 + 1;
  return g;
}

double p_unit(const edf_physics& P) { return P.rho0 * std::max(P.g, 1.0) * P.lz; }

Phys make_phys(const edf_physics& P, const Geom& g, double dt) {
  Phys ph{};
  ph.rho0 = P.rho0;
  ph.drho = P.rho1 - P.rho0;
  ph.mu = P.mu;
  ph.g = P.g;
  ph.Dm = P.Dm;
  ph.dt = dt;
  ph.row_c = 1.0 / (P.rho0 * P.phi_mean * g.hx * g.hy * g.hz);
  ph.s_row = dt * ph.row_c;
  ph.p_unit = p_unit(P);
  return ph;
}

// Newton also stops once the root-mean-square scaled update falls below this value:
// the unknowns are O(1) in scaled units, so further iterations only move rounding.
constexpr double kUpdateFloor = 1e-14;

// the V-cycle runs in FP32 (EDF_PREC_MIXED, EDF_PREC_MIXED_F16)
bool mixed(const edf_problem* pb) { return pb->opts.precision != EDF_PREC_F64; }
// the finest level's V-cycle matrix is stored in FP16 (it must be a smoothed level)
bool f16_finest(const edf_problem* pb, const Group& G) {
  return pb->opts.precision == EDF_PREC_MIXED_F16 && G.L >= 2;
}

constexpr int kFirstWait = 3, kMaxWait = 64;

// forget every sample's sub-step history (opts.substep_memory)
void reset_history(Group& G) {
  G.h_start.assign(G.S, 0);
  G.clean.assign(G.S, 0);
  G.wait.assign(G.S, kFirstWait);
  G.probing.assign(G.S, 0);
  G.pred_dt.assign(G.S, 0.0);
}

// ---------------------------------------------------------------------------
// allocation of one group
// ---------------------------------------------------------------------------
// Slots of the shared V-cycle allocations: for every grid, the groups that have a level
// on it, ordered by decreasing finest grid (then by group index), take consecutive slots.
// A group with a level on a grid has levels on every coarser grid of its hierarchy, so the
// groups of a grid come first on the next coarser one: a group's samples then have the
// same slots on consecutive levels whenever the groups' hierarchies are nested, which the
// merged restriction and prolongation need (it is checked before merging).
void plan_pools(edf_problem* pb) {
  std::map<std::tuple<int, int, int>, std::vector<int>> parts;
  const int ng = (int)pb->groups.size();
  for (int gi = 0; gi < ng; ++gi) {
    Group& G = pb->groups[gi];
    G.slots.assign(G.L, 0);
    int nx = G.d.nx, ny = G.d.ny, nz = G.d.nz;
    for (int l = 0; l < G.L; ++l) {
      parts[{nx, ny, nz}].push_back(gi);
      nx = (nx - 1) / 2 + 1;
      ny = (ny - 1) / 2 + 1;
      nz = (nz - 1) / 2 + 1;
    }
  }
  for (auto& kv : parts) {
    std::vector<int>& v = kv.second;
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
      const edf_group_desc &da = pb->groups[a].d, &db = pb->groups[b].d;
      return (long long)da.nx * da.ny * da.nz > (long long)db.nx * db.ny * db.nz;
    });
    int off = 0;
    for (int gi : v) {
      Group& G = pb->groups[gi];
      int nx = G.d.nx, ny = G.d.ny, nz = G.d.nz;
      for (int l = 0; l < G.L; ++l) {
        if (std::make_tuple(nx, ny, nz) == kv.first) G.slots[l] = off;
        nx = (nx - 1) / 2 + 1;
        ny = (ny - 1) / 2 + 1;
        nz = (nz - 1) / 2 + 1;
      }
      off += G.S;
    }
    pb->pool_slots[kv.first] = off;
  }
}

// the array of `kind` (bytes per sample) of level l of G, in its grid's shared allocation
edf_status take(edf_problem* pb, const Group& G, int l, int kind, size_t bytes, char** out) {
  const Geom& g = G.lv[l].g;
  for (const edf_problem::Pool& P : pb->pools)
    if (P.nx == g.nx && P.ny == g.ny && P.nz == g.nz && P.kind == kind) {
      if (P.per_sample != bytes) return fail(pb, EDF_ERR_STATE, "shared allocation size mismatch");
      *out = P.base + (size_t)G.lv[l].slot * bytes;
      return EDF_OK;
    }
  const size_t slots = pb->pool_slots[std::make_tuple(g.nx, g.ny, g.nz)];
  char* q;
  edf_status s;
  if ((s = dalloc(pb, &q, slots * bytes))) return s;
  pb->pools.push_back({g.nx, g.ny, g.nz, kind, bytes, q});
  *out = q + (size_t)G.lv[l].slot * bytes;
  return EDF_OK;
}

edf_status alloc_group(edf_problem* pb, Group& G) {
  const edf_physics& P = pb->phys;
  const int S = G.S;
  const bool mx = mixed(pb);
  const size_t tsz = mx ? sizeof(float) : sizeof(double);
  G.lv.resize(G.L);
  G.min_fuse = f16_finest(pb, G) ? 1 : 0;
  int nx = G.d.nx, ny = G.d.ny, nz = G.d.nz;
  for (int l = 0; l < G.L; ++l) {
    Level& L = G.lv[l];
    L.g = make_geom(nx, ny, nz, P);
    L.cells = (size_t)(nx - 1) * (ny - 1) * (nz - 1);
    const size_t N = L.g.N, Np = L.g.off[8];
    edf_status s;
    L.slot = G.slots[l];
    if ((s = dalloc(pb, &L.phi, S * L.cells))) return s;
    if ((s = dalloc(pb, &L.K, S * L.cells))) return s;
    if (l > 0 && (s = dalloc(pb, &L.u, S * 2 * N))) return s;
    const bool coarsest = l == G.L - 1;
    // level 0: the exact Jacobian of the Krylov products, unless they are matrix-free
    // (the adjoint allocates it when it needs the transposed products)
    if (l == 0 && !pb->opts.matrix_free)
      if ((s = dalloc(pb, &L.A64, S * kPlanes * Np))) return s;
    // the V-cycle arrays: in the shared allocations of the level's grid
    char* q;
    if (l > 0 && (!mx || coarsest)) {
      if ((s = take(pb, G, l, kPoolVA64, kPlanes * Np * sizeof(double), &q))) return s;
      L.A64 = reinterpret_cast<double*>(q);
    }
    if (mx && !coarsest) {
      if ((s = take(pb, G, l, kPoolA32, kPlanes * Np * sizeof(float), &q))) return s;
      L.A32 = reinterpret_cast<float*>(q);
    }
    if (l == 0 && f16_finest(pb, G))
      if ((s = dalloc(pb, &L.A16, S * kPlanes * Np))) return s;
    if (l == 0 && (!mx || coarsest)) {
      if ((s = take(pb, G, l, kPoolVA64, kPlanes * Np * sizeof(double), &q))) return s;
      L.AV64 = reinterpret_cast<double*>(q);
    }
    if (!coarsest) {
      if ((s = take(pb, G, l, kPoolDinv, 4 * Np * tsz, &q))) return s;
      L.Dinv = q;
      if (pb->opts.smoother == 1) {
        if ((s = take(pb, G, l, kPoolLF, kLineFactors * Np * tsz, &q))) return s;
        L.LF = q;
      }
      if ((s = take(pb, G, l, kPoolR, 2 * Np * tsz, &q))) return s;
      L.r = q;
    }
    if ((s = take(pb, G, l, kPoolB, 2 * Np * tsz, &q))) return s;
    L.b = q;
    if ((s = take(pb, G, l, kPoolX, 2 * Np * tsz, &q))) return s;
    L.x = q;
    nx = (nx - 1) / 2 + 1;
    ny = (ny - 1) / 2 + 1;
    nz = (nz - 1) / 2 + 1;
  }
  G.N = G.lv[0].g.N;
  G.n = 2 * G.N;
  const size_t n = G.n;
  edf_status s;
  double** vecs[] = {&G.u,  &G.u_old, &G.F,  &G.Ft, &G.ut,  &G.kx,  &G.kr,
                     &G.krh, &G.kp,   &G.kv, &G.ks_, &G.kt, &G.kph, &G.ksh};
  for (double** v : vecs)
    if ((s = dalloc(pb, v, S * n))) return s;
  G.lv[0].u = G.u;
  if ((s = dalloc(pb, &G.ks, (size_t)S))) return s;
  const size_t nb = std::max<size_t>(
      {(size_t)reduce_blocks(n), (size_t)ceil_div(G.lv[0].g.off[8], kBlock),
       (size_t)jx_blocks(G.lv[0].g)});
  if ((s = dalloc(pb, &G.part, S * nb * 4))) return s;
  if ((s = dalloc(pb, &G.nmask, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.active, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.d_list, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.lsmask, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.norms, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.lam, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.dts, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.eta, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.crange, 2 * (size_t)S))) return s;
  if ((s = dalloc(pb, &G.u0, S * n))) return s;
  if (pb->opts.predictor && (s = dalloc(pb, &G.u_prev, S * n))) return s;
  {
    char* q;
    if ((s = dalloc(pb, &q, sizeof(FusedLevels<double>)))) return s;
    G.fdesc = q;
  }
  G.n_coarse = 2 * G.lv[G.L - 1].g.N;
  const size_t nc = G.n_coarse;
  {
    char* q;
    if ((s = take(pb, G, G.L - 1, kPoolMinv, nc * nc * sizeof(double), &q))) return s;
    G.Minv = reinterpret_cast<double*>(q);
  }
  if ((s = dalloc(pb, &G.piv, S * nc))) return s;
  if ((s = dalloc(pb, &G.gj_status, (size_t)S))) return s;
  if ((s = dalloc(pb, &G.bal, 8 * (size_t)S))) return s;
  if ((s = dalloc(pb, &G.bal_part, 8 * (size_t)S * balance_blocks(G.lv[0].g)))) return s;
  G.stats.assign(S, edf_step_stats{});
  G.fail_status.assign(S, EDF_SAMPLE_OK);
  reset_history(G);
  return EDF_OK;
}

// initial state: p = rho0 g z, c = 1 on the patch, 0 elsewhere (host-built, uploaded)
edf_status upload_initial(edf_problem* pb, Group& G) {
  const Geom& g = G.lv[0].g;
  std::vector<double> u(G.n);
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const size_t v = i + (size_t)g.nx * (j + (size_t)g.ny * k);
        u[2 * v] = pb->phys.rho0 * pb->phys.g * k * g.hz;
        const bool patch = k == 0 && i >= g.pi0 && i <= g.pi1 && j >= g.pj0 && j <= g.pj1;
        u[2 * v + 1] = patch ? 1.0 : 0.0;
      }
  for (int s = 0; s < G.S; ++s) {
    EDF_TRY(hipMemcpyAsync(G.u + s * G.n, u.data(), G.n * sizeof(double), hipMemcpyHostToDevice,
                           G.st));
    EDF_TRY(hipMemcpyAsync(G.u_old + s * G.n, u.data(), G.n * sizeof(double),
                           hipMemcpyHostToDevice, G.st));
  }
  EDF_TRY(hipStreamSynchronize(G.st));
  return EDF_OK;
}

edf_status find_sample(edf_problem* pb, int sample, Group** G, int* local) {
  for (Group& g : pb->groups)
    if (sample >= g.s0 && sample < g.s0 + g.S) {
      *G = &g;
      *local = sample - g.s0;
      return EDF_OK;
    }
  return fail(pb, EDF_ERR_ARG, "sample index out of range");
}

// the vertical-line smoother's column factors of a level's V-cycle matrix (if it has any)
void line_factors(Level& L, bool mixed_vcycle, int S, const int* mask, hipStream_t st) {
  if (!L.LF) return;
  if (L.A16)  // FP16 finest level: the columns of the scaled matrix D^{-1} A
    launch_line_factor_f16(L.g, L.A16, (float*)L.LF, S, mask, st);
  else if (mixed_vcycle)
    launch_line_factor<float>(L.g, L.A32, (float*)L.LF, S, mask, st);
  else
    launch_line_factor<double>(L.g, L.AV64 ? L.AV64 : L.A64, (double*)L.LF, S, mask, st);
}

// ---------------------------------------------------------------------------
// matrices of all levels at the current iterate
// ---------------------------------------------------------------------------
edf_status assemble_all(edf_problem* pb, Group& G, const int* mask, const double* dts) {
  const bool mx = mixed(pb);
  G.transposed = false;
  for (int l = 0; l < G.L; ++l) {
    Level& L = G.lv[l];
    if (l > 0) launch_inject(G.lv[l - 1].g, L.g, G.lv[l - 1].u, L.u, G.S, mask, G.st);
    const bool coarsest = l == G.L - 1;
    if (l == 0 && L.A64 && !pb->opts.matrix_free)  // exact Jacobian for the Krylov products
      launch_assemble(L.g, L.ph, dts, L.phi, L.K, L.u, L.A64, nullptr, G.S, mask, G.st, false);
    // preconditioner matrix (frozen Darcy flux in the salt rows): FP32 on the smoothed
    // levels in mixed mode, FP64 otherwise and always on the coarsest level
    double* m64 = (mx && !coarsest) ? nullptr : (l == 0 ? L.AV64 : L.A64);
    float* m32 = (mx && !coarsest) ? L.A32 : nullptr;
    launch_assemble(L.g, L.ph, dts, L.phi, L.K, L.u, m64, m32, G.S, mask, G.st, true);
    if (!coarsest) {
      if (l == 0 && f16_finest(pb, G))
        launch_scale_f16(L.g, L.A32, L.A16, (float*)L.Dinv, G.S, mask, G.st);
      else if (mx)
        launch_block_inverse_f32(L.g, L.A32, (float*)L.Dinv, G.S, mask, G.st);
      else
        launch_block_inverse_f64(L.g, m64, (double*)L.Dinv, G.S, mask, G.st);
      line_factors(L, mx, G.S, mask, G.st);
    }
  }
  const Level& C = G.lv[G.L - 1];
  launch_coarse_dense(C.g, G.L == 1 ? C.AV64 : C.A64, G.Minv, G.S, mask, G.st);
  launch_gauss_jordan(G.n_coarse, G.Minv, G.piv, G.gj_status, G.S, mask, G.st);
  EDF_CHECK_LAUNCH();
  return EDF_OK;
}

// ---------------------------------------------------------------------------
// smoother timing
// ---------------------------------------------------------------------------
// every kProfStride-th smoother launch is timed (events around every launch would
// themselves cost about a tenth of the run time); 13 is coprime with the 8 colours
// and 16 launches of a pre- and post-smoothing pair
constexpr int kProfStride = 13;

bool prof_pair(Group& G, hipEvent_t& a, hipEvent_t& b, double bytes, int kind) {
  if (!G.prof_on) return false;
  const bool large = bytes > kLargeLaunch;
  if (kind == 0) {
    G.prof_all_count[0] += 1;
    G.prof_all_bytes[0] += bytes;
    if (large) {
      G.prof_all_count[1] += 1;
      G.prof_all_bytes[1] += bytes;
    }
    if (G.prof_tick++ % kProfStride != 0) return false;
  }
  const size_t k = G.prof_pending.size();
  while (G.prof_ev.size() < 2 * (k + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    G.prof_ev.push_back(e);
  }
  a = G.prof_ev[2 * k];
  b = G.prof_ev[2 * k + 1];
  G.prof_pending.push_back({(int)k, kind, bytes, large});
  return true;
}

edf_status prof_flush(edf_problem* pb, Group& G) {
  for (auto& r : G.prof_pending) {
    float ms = 0.f;
    EDF_TRY(hipEventSynchronize(G.prof_ev[2 * r.pair + 1]));
    EDF_TRY(hipEventElapsedTime(&ms, G.prof_ev[2 * r.pair], G.prof_ev[2 * r.pair + 1]));
    G.prof_count[r.kind] += 1;
    G.prof_ms[r.kind] += ms;
    G.prof_bytes[r.kind] += r.bytes;
    if (r.large) {  // [2]: smoother launches, [3]: V-cycles beyond the last-level cache
      const int q = r.kind == 0 ? 2 : 3;
      G.prof_count[q] += 1;
      G.prof_ms[q] += ms;
      G.prof_bytes[q] += r.bytes;
    }
  }
  G.prof_pending.clear();
  return EDF_OK;
}

// algorithmic bytes of one V-cycle per sample: on every smoothed level, nu1 + nu2 + 1
// stencil sweeps (smoothing sweeps and the residual), nu1 + nu2 block-inverse reads
// and 3 (nu1 + nu2) + 6 vector passes (b, x in and x out per smoothing sweep; b, x
// in and r out for the residual; r into the restriction; x in and out for the
// correction), plus the coarse right-hand side and solution and the dense inverse
static_assert(zero_start_blocks(0) == 0 && zero_start_blocks(7) == 26, "zero-start stencil reads");
static_assert(zero_start_blocks(0) + zero_start_blocks(1) + zero_start_blocks(2) +
                      zero_start_blocks(3) + zero_start_blocks(4) + zero_start_blocks(5) +
                      zero_start_blocks(6) + zero_start_blocks(7) ==
                  8 * 13,
              "each off-diagonal coupling is read from one of its two ends");

// Algorithmic bytes per vertex of colour c of one smoother sweep.  A sweep reads the 27
// stencil blocks, the block inverse, b and the vertex's own x and writes x (118 values);
// the first forward sweep from x = 0 reads only the blocks of the colours already swept,
// the block inverse and b, and writes x.  FP16 finest level: the 26 off-diagonal FP16
// blocks, D^{-1} b, x in and out (FP32), from zero the swept colours' blocks, D^{-1} b
// and x out.
double sweep_bytes(int c, bool zero_start, bool fp16, size_t tsz) {
  const int nb = zero_start_blocks(c);
  if (fp16) return zero_start ? nb * 4 * 2 + 4 * 4 : 26 * 4 * 2 + 6 * 4;
  return (zero_start ? 4.0 * nb + 8.0 : kPlanes + 10.0) * tsz;
}

// Algorithmic bytes per vertex of column colour cc of one vertical-line sweep: the
// stencil blocks towards the other columns (24, or from zero the 3 per column of the
// colours already swept) and the block above, the column factors (8 values), b, and x
// written three times over (the forward pass stores d in x, the backward pass reads it
// and writes x).
double line_sweep_bytes(int cc, bool zero_start, size_t tsz) {
  const int nb = zero_start ? line_zero_start_blocks(cc) : 24;
  return (4.0 * (nb + 1) + 8 + 2 + 6) * tsz;
}
// the residual after a single forward line sweep from zero: the blocks towards the
// columns of the colours swept later, and r
double line_residual_bytes(int cc, size_t tsz) {
  return (4.0 * (24 - line_zero_start_blocks(cc)) + 2) * tsz;
}
// FP16-stored finest level: 8 bytes per 2x2 block, the FP32 factors, D^{-1} b and x (FP32);
// its residual also reads the FP32 diagonal blocks D to unscale
double line_sweep_bytes_f16(int cc, bool zero_start) {
  const int nb = zero_start ? line_zero_start_blocks(cc) : 24;
  return 8.0 * (nb + 1) + (8 + 2 + 6) * 4.0;
}
double line_residual_bytes_f16(int cc) {
  return 8.0 * (24 - line_zero_start_blocks(cc)) + (4 + 2) * 4.0;
}
static_assert(line_zero_start_blocks(0) == 0 && line_zero_start_blocks(1) == 6 &&
                  line_zero_start_blocks(2) == 18 && line_zero_start_blocks(3) == 24,
              "each coupling between columns is read from one of its two ends");

// Algorithmic bytes of one V-cycle per sample: on every level above the coarsest, the
// nu1 + nu2 sweeps (the first forward one from zero), the residual (stencil, b, x in,
// r out; after a single sweep from zero only the blocks towards the colours swept later
// and r out), r into the restriction and x in and out for the correction; then the dense
// coarse inverse and its vectors.
double vcycle_bytes(const Group& G, size_t tsz, int nu1, int nu2, int l0) {
  const bool zs_res = nu1 == 1 && !G.transposed;
  double b = 0;
  for (int l = 0; l + 1 < G.L; ++l) {
    const Geom& g = G.lv[l].g;
    const bool h = l == 0 && G.lv[0].A16;
    if (G.lv[l].LF && l < l0) {  // vertical-line smoothing
      auto sweep = [&](int cc, bool zs) {
        return h ? line_sweep_bytes_f16(cc, zs) : line_sweep_bytes(cc, zs, tsz);
      };
      for (int cc = 0; cc < 4; ++cc) {
        const double nv = (double)g.mx[cc] * g.my[cc] * g.nz;
        b += nv * ((nu1 + nu2) * sweep(cc, false));
        if (nu1 > 0) b += nv * (sweep(cc, true) - sweep(cc, false));
        if (h)  // the residual reads the FP16 blocks, D, D^{-1} b and x (general) or the
                // blocks towards the later columns and D (after one sweep from zero)
          b += nv * (zs_res ? line_residual_bytes_f16(cc) : (26 * 4 * 2 + 4 * 4 + 6 * 4 + 2 * 4));
        else
          b += nv * (zs_res ? line_residual_bytes(cc, tsz) : (kPlanes + 12.0) * tsz);
      }
      continue;
    }
    for (int c = 0; c < 8; ++c)
      b += (double)g.cnt[c] * (nu1 * sweep_bytes(c, false, h, tsz) + nu2 * sweep_bytes(c, false, h, tsz));
    if (nu1 > 0)
      for (int c = 0; c < 8; ++c)
        b += (double)g.cnt[c] * (sweep_bytes(c, true, h, tsz) - sweep_bytes(c, false, h, tsz));
    if (h && zs_res) {  // FP16 blocks towards the later colours, D (FP32), r out
      for (int c = 0; c < 8; ++c)
        b += (double)g.cnt[c] * ((26 - zero_start_blocks(c)) * 4 * 2 + 4 * 4 + 2 * 4 + 2 * 4 + 4 * 4);
    } else if (h) {  // the residual reads the FP16 blocks, D (FP32), D^{-1} b and x and writes r
      b += (double)g.N * ((26 * 4 * 2 + 4 * 4 + 6 * 4) + 2 * 4 + 4 * 4);
    } else if (zs_res) {
      for (int c = 0; c < 8; ++c)
        b += (double)g.cnt[c] * (4.0 * (26 - zero_start_blocks(c)) + 8.0) * tsz;
    } else {
      b += (double)g.N * (kPlanes + 12.0) * tsz;
    }
  }
  const double nc = G.n_coarse;
  return b + nc * nc * 8.0 + 2.0 * nc * tsz;
}

// ---------------------------------------------------------------------------
// one V-cycle: out = M^{-1} in (FP64 vectors of the scaled unknowns)
// ---------------------------------------------------------------------------
// The V-cycle's sample list: the samples s with flags[s] != 0, in order.  Called with the
// group's stream idle (after a synchronisation), so the pinned copy feeds no pending copy.
edf_status set_sample_list(edf_problem* pb, Group& G, const int* flags) {
  int n = 0;
  bool same = true;
  for (int s = 0; s < G.S; ++s)
    if (flags[s]) {
      same = same && n < G.n_list && G.h_list[n] == s;
      G.h_list[n++] = s;
    }
  if (same && n == G.n_list) return EDF_OK;
  G.n_list = n;
  ++G.list_ver;
  if (n > 0)
    EDF_TRY(hipMemcpyAsync(G.d_list, G.h_list, n * sizeof(int), hipMemcpyHostToDevice, G.st));
  return EDF_OK;
}

// first level of the fused bottom of the V-cycle when not tuned: all levels of at
// most kFuseMaxN vertices when the group has many samples (their workgroups run side
// by side), else only the coarse solve (one workgroup per sample walks the levels
// one after the other, which does not pay for a single sample)
int first_fusable(const Group& G) {
  int l0 = G.L - 1;
  while (l0 > G.min_fuse && G.lv[l0 - 1].g.N <= kFuseMaxN && G.L - l0 < kMaxFused) --l0;
  return l0;
}
int default_fuse_from(const Group& G) { return G.S >= 64 ? first_fusable(G) : G.L - 1; }

template <typename T>
const T* stencil(const Level& L);
template <>
const double* stencil<double>(const Level& L) { return L.AV64 ? L.AV64 : L.A64; }
template <>
const float* stencil<float>(const Level& L) { return L.A32; }

// the fused bottom's description for first fused level l0 (host side), whether the
// levels' vectors fit in the workgroup's LDS, and the dynamic LDS of its launch: the
// vectors when they fit, and the values of one line sweep of the largest line-smoothed
// level (levels with line factors are swept by lines, as those swept by their own
// launches; point sweeps if even those values do not fit)
template <typename T>
FusedLevels<T> fused_levels(const Group& G, int l0, size_t& lds_bytes, bool& in_lds) {
  FusedLevels<T> F{};
  F.n = G.L - l0;
  F.nc = G.n_coarse;
  F.Minv = G.Minv;
  // the levels' x, b and r (three vectors of 2 Np_k) in LDS when they all fit
  size_t lds_elems = 0, scr = 0;
  for (int k = 0; k < F.n; ++k) {
    const Level& L = G.lv[l0 + k];
    F.g[k] = L.g;
    const bool coarsest = l0 + k == G.L - 1;
    F.A[k] = coarsest ? nullptr : stencil<T>(L);
    F.D[k] = coarsest ? nullptr : (const T*)L.Dinv;
    F.LF[k] = coarsest || L.A16 ? nullptr : (const T*)L.LF;
    F.r[k] = coarsest ? nullptr : (T*)L.r;
    F.b[k] = (T*)L.b;
    F.x[k] = (T*)L.x;
    F.lds_off[k] = (int)lds_elems;
    lds_elems += 6 * (size_t)L.g.off[8];
    if (F.LF[k]) {
      int most = 0;
      for (int cc = 0; cc < 4; ++cc) most = std::max(most, L.g.mx[cc] * L.g.my[cc]);
      scr = std::max(scr, (size_t)kLineVals * L.g.nz * most);
    }
  }
  const size_t limit = vcycle_bottom_lds_limit<T>();
  in_lds = (lds_elems + scr) * sizeof(T) <= limit;
  if (in_lds) {
    F.line_lds = scr ? (int)lds_elems : -1;
    lds_bytes = (lds_elems + scr) * sizeof(T);
  } else {
    for (int k = 0; k < F.n; ++k) F.lds_off[k] = -1;
    F.line_lds = scr && scr * sizeof(T) <= limit ? 0 : -1;
    lds_bytes = F.line_lds == 0 ? scr * sizeof(T) : 0;
  }
  return F;
}

// the device copy of the description; it changes only with the first fused level (and
// the smoothing counts, fixed per problem)
template <typename T>
void ensure_fused_desc(edf_problem* pb, Group& G, int l0) {
  if (G.fdesc_l0 == l0) return;
  size_t lds_bytes;
  bool in_lds;
  FusedLevels<T> F = fused_levels<T>(G, l0, lds_bytes, in_lds);
  F.nu1 = pb->opts.nu_pre;
  F.nu2 = pb->opts.nu_post;
  (void)hipMemcpyAsync(G.fdesc, &F, sizeof(F), hipMemcpyHostToDevice, G.st);
  (void)hipStreamSynchronize(G.st);
  G.fdesc_l0 = l0;
}

int first_fused_level(const Group& G) {
  return G.fuse_from >= 0 ? G.fuse_from : default_fuse_from(G);
}

template <typename T>
void vcycle(edf_problem* pb, Group& G, const double* in, double* out, const int* mask) {
  hipStream_t st = G.st;
  // launches run over the listed samples (mask still decides exactness); no list when it
  // holds every sample
  const int S = G.n_list;
  const int* list = G.n_list < G.S ? G.d_list : nullptr;
  if (S == 0) return;
  const int nu1 = pb->opts.nu_pre, nu2 = pb->opts.nu_post;
  T* b0 = (T*)G.lv[0].b;
  T* x0 = (T*)G.lv[0].x;
  // residual from the blocks towards the later colours after a single zero-start sweep
  // (equal to b - A x in exact arithmetic); the adjoint's transposed systems keep b - A x
  const bool zs_res = nu1 == 1 && !G.transposed;
  // finest level with an FP16 matrix: b0 holds D^{-1} b (only for T = float)
  const bool h0 = std::is_same<T, float>::value && G.L >= 2 && G.lv[0].A16;
  const int l0 = first_fused_level(G);
  // vertical-line smoothing on the levels swept by their own launches that have factors
  auto line = [&](int l) { return l < l0 && G.lv[l].LF != nullptr; };
  // the first forward sweep from zero of colour 0 (x = D^{-1} b, no neighbours) is done by
  // the kernel that writes the level's b: the entry permutation here, the restriction on
  // the coarser levels swept by separate point-smoother launches
  const bool c0 = nu1 > 0;
  const bool c0_here = c0 && l0 > 0 && !line(0);
  if constexpr (std::is_same<T, float>::value) {
    if (h0)
      launch_to_colour_scaled(G.lv[0].g, in, (const float*)G.lv[0].Dinv, (float*)b0,
                              c0_here ? (float*)x0 : nullptr, S, mask, list, st);
    else
      launch_to_colour<T>(G.lv[0].g, in, b0, c0_here ? (const T*)G.lv[0].Dinv : nullptr, x0, S,
                          mask, list, st);
  } else {
    launch_to_colour<T>(G.lv[0].g, in, b0, c0_here ? (const T*)G.lv[0].Dinv : nullptr, x0, S,
                        mask, list, st);
  }
  // zs: the first forward sweep of the level, whose x is zero on entry
  auto smooth = [&](int l, const Level& L, int c, const T* b, T* x, bool zs) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (line(l)) {
      const double nv = (double)L.g.mx[c] * L.g.my[c] * L.g.nz;
      if constexpr (std::is_same<T, float>::value) {
        if (l == 0 && h0) {  // FP16 blocks of the scaled system, b = D^{-1} b
          prof_pair(G, e0, e1, nv * G.n_active * line_sweep_bytes_f16(c, zs), 0);
          launch_line_smooth_f16(L.g, c, L.A16, (const float*)L.LF, (const float*)b, (float*)x, S,
                                 mask, list, st, e0, e1, zs, L.line_cols);
          return;
        }
      }
      prof_pair(G, e0, e1, nv * G.n_active * line_sweep_bytes(c, zs, sizeof(T)), 0);
      launch_line_smooth<T>(L.g, c, stencil<T>(L), (const T*)L.LF, b, x, S, mask, list, st, e0,
                            e1, zs, L.line_cols);
      return;
    }
    const double per_vertex = sweep_bytes(c, zs, l == 0 && h0, sizeof(T));
    prof_pair(G, e0, e1, (double)L.g.cnt[c] * G.n_active * per_vertex, 0);
    if constexpr (std::is_same<T, float>::value) {
      if (l == 0 && h0) {
        launch_smooth_f16(L.g, c, L.A16, (const float*)b, (float*)x, S, mask, list, st, e0, e1, zs);
        return;
      }
    }
    launch_smooth<T>(L.g, c, stencil<T>(L), (const T*)L.Dinv, b, x, S, mask, list, st, e0, e1, zs);
  };
  auto residual = [&](int l, const Level& L, const T* b, const T* x) {
    if constexpr (std::is_same<T, float>::value) {
      if (l == 0 && h0) {
        if (line(l) && zs_res)  // after one line sweep from zero: the later columns' blocks
          launch_line_residual_zs_f16(L.g, L.A16, (const float*)L.Dinv, (const float*)x,
                                      (float*)L.r, S, mask, list, st);
        else  // general r = D (D^{-1} b - A16 x), or after one point sweep from zero
          launch_residual_f16(L.g, L.A16, (const float*)L.Dinv, (const float*)b, (const float*)x,
                              (float*)L.r, S, mask, list, st, zs_res && !line(l));
        return;
      }
    }
    if (line(l) && zs_res) {
      launch_line_residual_zs<T>(L.g, stencil<T>(L), x, (T*)L.r, S, mask, list, st);
      return;
    }
    launch_residual<T>(L.g, stencil<T>(L), b, x, (T*)L.r, S, mask, list, st, zs_res && !line(l));
  };
  auto bx = [&](int l, T*& b, T*& x) {
    b = l == 0 ? b0 : (T*)G.lv[l].b;
    x = l == 0 ? x0 : (T*)G.lv[l].x;
  };
  // levels from l0 on run in one fused launch (one workgroup per sample)
  // every level starts from x = 0: the first forward sweep writes x at every vertex
  // without reading it, so x needs clearing only without pre-smoothing
  if (l0 > 0 && nu1 == 0) launch_fill<T>(x0, 2 * (size_t)G.lv[0].g.off[8], G.S, mask, T(0), st);
  for (int l = 0; l < l0; ++l) {
    Level& L = G.lv[l];
    T *b, *x;
    bx(l, b, x);
    const int ncol = line(l) ? 4 : 8;
    for (int it = 0; it < nu1; ++it)
      for (int c = it == 0 && c0 && !line(l) ? 1 : 0; c < ncol; ++c) smooth(l, L, c, b, x, it == 0);
    residual(l, L, b, x);
    T *bc, *xc;
    bx(l + 1, bc, xc);
    // x of the next level needs no clearing when its first sweep starts from zero (for a
    // point-smoothed level its colour 0 done here) or when it is the fused bottom's first
    // level (cleared there)
    const bool next_swept = l + 1 < l0;
    const bool next_point = next_swept && !line(l + 1);
    launch_restrict<T>(L.g, G.lv[l + 1].g, (const T*)L.r, bc,
                       c0 ? (next_point ? xc : nullptr) : xc,
                       c0 && next_point ? (const T*)G.lv[l + 1].Dinv : nullptr, S, mask, list, st);
  }
  {
    size_t lds_bytes = 0;
    bool in_lds = false;
    (void)fused_levels<T>(G, l0, lds_bytes, in_lds);
    ensure_fused_desc<T>(pb, G, l0);  // a no-op inside a captured V-cycle (set up before)
    launch_vcycle_bottom<T>((const FusedLevels<T>*)G.fdesc, lds_bytes, S, mask, list, st);
  }
  for (int l = l0 - 1; l >= 0; --l) {
    Level& L = G.lv[l];
    T *b, *x, *bc, *xc;
    bx(l, b, x);
    bx(l + 1, bc, xc);
    launch_prolong<T>(L.g, G.lv[l + 1].g, xc, x, S, mask, list, st);
    const int ncol = line(l) ? 4 : 8;
    for (int it = 0; it < nu2; ++it)
      for (int c = ncol - 1; c >= 0; --c) smooth(l, L, c, b, x, false);
  }
  launch_from_colour<T>(G.lv[0].g, x0, out, S, mask, list, st);
}

// The V-cycle as a captured graph: the same launches in the same order, replayed with one
// graph launch.  A graph is captured the first time a launch configuration (first fused
// level, number of listed samples, residual form, vectors) occurs and replayed after; the
// kernels read the matrices, the sample list and the fused description at replay, so
// reassembly and new lists need no new capture.  False when capturing fails (the caller
// then runs the V-cycle eagerly).
template <typename T>
bool vcycle_graph(edf_problem* pb, Group& G, const double* in, double* out, const int* mask) {
  const int l0 = first_fused_level(G);
  ensure_fused_desc<T>(pb, G, l0);  // outside the capture: it copies and synchronises
  const int listed = G.n_list < G.S, zs = pb->opts.nu_pre == 1 && !G.transposed;
  for (const auto& v : G.vgraphs)
    if (v.l0 == l0 && v.n_list == G.n_list && v.listed == listed && v.zs == zs && v.in == in &&
        v.out == out && v.mask == mask)
      return hipGraphLaunch(v.exec, G.st) == hipSuccess;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(G.st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  vcycle<T>(pb, G, in, out, mask);
  if (hipStreamEndCapture(G.st, &graph) != hipSuccess || !graph) {
    (void)hipGetLastError();
    return false;
  }
  hipGraphExec_t exec = nullptr;
  const bool ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(graph);
  if (!ok) {
    (void)hipGetLastError();
    return false;
  }
  G.vgraphs.push_back({l0, G.n_list, listed, zs, in, out, mask, exec});
  return hipGraphLaunch(exec, G.st) == hipSuccess;
}

// ---------------------------------------------------------------------------
// merged V-cycles (concurrent_groups = 2): the V-cycles of several groups in one pass,
// every level that groups share (same grid, same role in the cycle) swept by one launch
// over all their listed samples.  The per-sample arithmetic is that of vcycle(): the
// same kernels on the same slots, so the results are bitwise those of separate cycles.
// ---------------------------------------------------------------------------
const int* sample_list(const Group& G) { return G.n_list < G.S ? G.d_list : nullptr; }

// start of a shared allocation, from a level's pointer into it
const char* pool_base(const void* p, int slot, size_t per_sample) {
  return p ? static_cast<const char*>(p) - (size_t)slot * per_sample : nullptr;
}

// one launch's list over the pairs (G, l): the slots of the groups' listed samples,
// rebuilt on the device when a group's list changed since the last use
const int* merged_list(edf_problem* pb, const std::vector<std::pair<Group*, int>>& parts,
                       int& rows, hipStream_t st) {
  std::vector<long> key, vkey;
  ListSegs L{};
  rows = 0;
  for (const auto& pr : parts) {
    Group* G = pr.first;
    key.push_back((long)(intptr_t)G);
    key.push_back(pr.second);
    vkey.push_back(G->list_ver);
    vkey.push_back(G->n_list);
    L.seg[L.nseg++] = {sample_list(*G), G->n_list, G->lv[pr.second].slot, rows};
    rows += G->n_list;
  }
  edf_problem::ListBuf* buf = nullptr;
  for (auto& b : pb->mg_lists)
    if (b.key == key) buf = &b;
  if (!buf) {
    const Geom& g = parts[0].first->lv[parts[0].second].g;
    int* d = nullptr;
    if (dalloc(pb, &d, (size_t)pb->pool_slots[std::make_tuple(g.nx, g.ny, g.nz)])) return nullptr;
    pb->mg_lists.push_back({key, {}, d, 0});
    buf = &pb->mg_lists.back();
  }
  if (buf->vkey != vkey) {
    launch_concat_lists(L, rows, buf->d, st);
    buf->vkey = vkey;
    buf->n = rows;
  }
  return buf->d;
}

template <typename T>
void vcycle_merged(edf_problem* pb, const std::vector<MergeReq*>& R) {
  std::vector<MergeReq*> W;
  for (MergeReq* r : R)
    if (r->G->n_list > 0) W.push_back(r);
  if (W.empty()) return;
  // cycles the merged pass does not cover run one by one: a single group, the adjoint's
  // transposed systems (general residual), an FP16 finest level, more than kMaxListSegs
  bool plain = W.size() == 1 || W.size() > (size_t)kMaxListSegs;
  for (MergeReq* r : W)
    plain = plain || r->G->transposed || (std::is_same<T, float>::value && r->G->lv[0].A16);
  if (plain) {
    for (MergeReq* r : W) {
      Group& G = *r->G;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const double bytes =
          vcycle_bytes(G, sizeof(T), pb->opts.nu_pre, pb->opts.nu_post, first_fused_level(G)) *
          G.n_active;
      if (prof_pair(G, e0, e1, bytes, 1)) (void)hipEventRecord(e0, G.st);
      vcycle<T>(pb, G, r->in, r->out, r->mask);
      if (e1) (void)hipEventRecord(e1, G.st);
    }
    return;
  }
  Group& G0 = *W[0]->G;
  hipStream_t st = G0.st;  // the groups share one stream in this mode
  const int nu1 = pb->opts.nu_pre, nu2 = pb->opts.nu_post;
  const bool zs_res = nu1 == 1;
  const bool c0 = nu1 > 0;
  const size_t tsz = sizeof(T);
  hipEvent_t ve0 = nullptr, ve1 = nullptr;
  {
    double bytes = 0;
    for (MergeReq* r : W)
      bytes += vcycle_bytes(*r->G, tsz, nu1, nu2, first_fused_level(*r->G)) * r->G->n_active;
    if (prof_pair(G0, ve0, ve1, bytes, 1)) (void)hipEventRecord(ve0, st);
  }
  auto l0of = [&](const Group* G) { return first_fused_level(*G); };
  auto line = [&](const Group* G, int l) { return l < l0of(G) && G->lv[l].LF != nullptr; };
  auto mask_of = [&](const Group* G) -> const int* {
    for (MergeReq* r : W)
      if (r->G == G) return r->mask;
    return nullptr;
  };
  // entry permutations (per group)
  for (MergeReq* r : W) {
    Group& G = *r->G;
    const int l0 = l0of(&G);
    const bool c0_here = c0 && l0 > 0 && !line(&G, 0);
    launch_to_colour<T>(G.lv[0].g, r->in, (T*)G.lv[0].b,
                        c0_here ? (const T*)G.lv[0].Dinv : nullptr, (T*)G.lv[0].x, G.n_list,
                        r->mask, sample_list(G), st);
  }
  // the swept levels, grouped by grid and role: (nx, ny, nz, line, next swept, next point)
  struct Station {
    std::tuple<int, int, int, int, int, int> key;
    long long N;
    std::vector<std::pair<Group*, int>> parts;
  };
  std::vector<Station> stations;
  for (MergeReq* r : W) {
    Group* G = r->G;
    for (int l = 0; l < l0of(G); ++l) {
      const Geom& g = G->lv[l].g;
      const bool ln = line(G, l), nsw = l + 1 < l0of(G), npt = nsw && !line(G, l + 1);
      auto key = std::make_tuple(g.nx, g.ny, g.nz, (int)ln, (int)nsw, (int)npt);
      Station* at = nullptr;
      for (Station& q : stations)
        if (q.key == key) at = &q;
      if (!at) {
        stations.push_back({key, (long long)g.N, {}});
        at = &stations.back();
      }
      at->parts.push_back({G, l});
    }
  }
  std::stable_sort(stations.begin(), stations.end(),
                   [](const Station& a, const Station& b) { return a.N > b.N; });
  // whether the pairs' arrays lie in common allocations at their slots (and their next
  // level's at the same slots), so that one launch over slots serves them all
  auto aligned = [&](const std::vector<std::pair<Group*, int>>& parts) {
    if (parts.size() < 2 || parts.size() > (size_t)kMaxListSegs) return false;
    const Level& A = parts[0].first->lv[parts[0].second];
    const Level& Ac = parts[0].first->lv[parts[0].second + 1];
    const size_t Np = A.g.off[8], Npc = Ac.g.off[8];
    for (const auto& pr : parts) {
      const Level& L = pr.first->lv[pr.second];
      const Level& Lc = pr.first->lv[pr.second + 1];
      if (L.slot != Lc.slot) return false;
      const int s = L.slot, a = A.slot;
      auto same = [&](const void* p, const void* q, size_t per) {
        return pool_base(p, s, per) == pool_base(q, a, per);
      };
      if (!same(stencil<T>(L), stencil<T>(A), kPlanes * Np * tsz) ||
          !same(L.Dinv, A.Dinv, 4 * Np * tsz) || !same(L.LF, A.LF, kLineFactors * Np * tsz) ||
          !same(L.b, A.b, 2 * Np * tsz) || !same(L.x, A.x, 2 * Np * tsz) ||
          !same(L.r, A.r, 2 * Np * tsz) || !same(Lc.b, Ac.b, 2 * Npc * tsz) ||
          !same(Lc.x, Ac.x, 2 * Npc * tsz) || !same(Lc.Dinv, Ac.Dinv, 4 * Npc * tsz))
        return false;
    }
    return true;
  };
  // a launch target: the arrays at slot 0 of the shared allocations (merged) or the
  // group's own arrays (one pair), the rows and list of the launch, active samples
  struct Target {
    const Level* L;
    const Level* Lc;
    const T* A;
    const T* F;
    const T* D;
    T *b, *x, *r, *bc, *xc;
    const T* Dc;
    int rows;
    const int* list;
    const int* mask;
    double active;
    bool ln, npt, nsw;
  };
  auto target = [&](const std::vector<std::pair<Group*, int>>& parts, bool merge) {
    std::vector<Target> out;
    auto one = [&](Group* G, int l, int slot, int rows, const int* list, const int* mask,
                   double active) {
      const Level& L = G->lv[l];
      const Level& Lc = G->lv[l + 1];
      const size_t Np = L.g.off[8], Npc = Lc.g.off[8];
      auto at = [&](const void* p, size_t per) {
        return p ? (char*)pool_base(p, L.slot, per) + (size_t)slot * per : nullptr;
      };
      auto atc = [&](const void* p, size_t per) {
        return p ? (char*)pool_base(p, Lc.slot, per) + (size_t)slot * per : nullptr;
      };
      Target t{&L, &Lc,
               (const T*)at(stencil<T>(L), kPlanes * Np * tsz),
               (const T*)at(L.LF, kLineFactors * Np * tsz),
               (const T*)at(L.Dinv, 4 * Np * tsz),
               (T*)at(L.b, 2 * Np * tsz), (T*)at(L.x, 2 * Np * tsz), (T*)at(L.r, 2 * Np * tsz),
               (T*)atc(Lc.b, 2 * Npc * tsz), (T*)atc(Lc.x, 2 * Npc * tsz),
               (const T*)atc(Lc.Dinv, 4 * Npc * tsz),
               rows, list, mask, active, line(G, l), false, l + 1 < l0of(G)};
      t.npt = t.nsw && !line(G, l + 1);
      out.push_back(t);
    };
    if (merge) {
      int rows = 0;
      const int* list = merged_list(pb, parts, rows, st);
      double active = 0;
      for (const auto& pr : parts) active += pr.first->n_active;
      // slot 0 of the shared allocations; the list holds slots; the groups' active flags
      // are not in slot order, so the listed samples (those active at the last count)
      // are all swept, as within a chunk of BiCGStab iterations
      one(parts[0].first, parts[0].second, 0, rows, list, nullptr, active);
    } else {
      for (const auto& pr : parts) {
        Group* G = pr.first;
        one(G, pr.second, G->lv[pr.second].slot, G->n_list, sample_list(*G), mask_of(G),
            (double)G->n_active);
      }
    }
    return out;
  };
  auto smooth = [&](const Target& t, int c, const T* b, T* x, bool zs) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const Geom& g = t.L->g;
    if (t.ln) {
      const double nv = (double)g.mx[c] * g.my[c] * g.nz;
      prof_pair(G0, e0, e1, nv * t.active * line_sweep_bytes(c, zs, tsz), 0);
      launch_line_smooth<T>(g, c, t.A, t.F, b, x, t.rows, t.mask, t.list, st, e0, e1, zs,
                            t.L->line_cols);
      return;
    }
    prof_pair(G0, e0, e1, (double)g.cnt[c] * t.active * sweep_bytes(c, zs, false, tsz), 0);
    launch_smooth<T>(g, c, t.A, t.D, b, x, t.rows, t.mask, t.list, st, e0, e1, zs);
  };
  std::vector<std::vector<Target>> plan(stations.size());
  for (size_t q = 0; q < stations.size(); ++q) {
    plan[q] = target(stations[q].parts, aligned(stations[q].parts));
    for (const Target& t : plan[q]) {
      const int ncol = t.ln ? 4 : 8;
      for (int it = 0; it < nu1; ++it)
        for (int c = it == 0 && c0 && !t.ln ? 1 : 0; c < ncol; ++c) smooth(t, c, t.b, t.x, it == 0);
      if (t.ln && zs_res)
        launch_line_residual_zs<T>(t.L->g, t.A, t.x, t.r, t.rows, t.mask, t.list, st);
      else
        launch_residual<T>(t.L->g, t.A, t.b, t.x, t.r, t.rows, t.mask, t.list, st,
                           zs_res && !t.ln);
      launch_restrict<T>(t.L->g, t.Lc->g, t.r, t.bc, c0 ? (t.npt ? t.xc : nullptr) : t.xc,
                         c0 && t.npt ? t.Dc : nullptr, t.rows, t.mask, t.list, st);
    }
  }
  // the fused bottoms: groups whose fused levels lie on the same grids share one launch
  {
    std::vector<std::vector<Group*>> classes;
    for (MergeReq* r : W) {
      Group* G = r->G;
      bool placed = false;
      for (auto& c : classes) {
        Group* H = c[0];
        const int a = l0of(G), b = l0of(H);
        bool same = G->L - a == H->L - b && c.size() < (size_t)kMaxListSegs;
        for (int k = 0; same && a + k < G->L; ++k) {
          const Level &X = G->lv[a + k], &Y = H->lv[b + k];
          const size_t Np = X.g.off[8];
          same = X.g.nx == Y.g.nx && X.g.ny == Y.g.ny && X.g.nz == Y.g.nz &&
                 X.slot == G->lv[a].slot && Y.slot == H->lv[b].slot &&
                 pool_base(X.b, X.slot, 2 * Np * tsz) == pool_base(Y.b, Y.slot, 2 * Np * tsz) &&
                 pool_base(X.x, X.slot, 2 * Np * tsz) == pool_base(Y.x, Y.slot, 2 * Np * tsz) &&
                 pool_base(X.r, X.slot, 2 * Np * tsz) == pool_base(Y.r, Y.slot, 2 * Np * tsz) &&
                 pool_base(X.Dinv, X.slot, 4 * Np * tsz) ==
                     pool_base(Y.Dinv, Y.slot, 4 * Np * tsz) &&
                 pool_base(X.LF, X.slot, kLineFactors * Np * tsz) ==
                     pool_base(Y.LF, Y.slot, kLineFactors * Np * tsz) &&
                 (a + k == G->L - 1 ||
                  pool_base(stencil<T>(X), X.slot, kPlanes * Np * tsz) ==
                      pool_base(stencil<T>(Y), Y.slot, kPlanes * Np * tsz));
        }
        const size_t nc2 = (size_t)G->n_coarse * G->n_coarse * sizeof(double);
        same = same && G->n_coarse == H->n_coarse &&
               pool_base(G->Minv, G->lv[G->L - 1].slot, nc2) ==
                   pool_base(H->Minv, H->lv[H->L - 1].slot, nc2);
        if (same) {
          c.push_back(G);
          placed = true;
          break;
        }
      }
      if (!placed) classes.push_back({G});
    }
    for (auto& c : classes) {
      Group* G = c[0];
      const int l0 = l0of(G);
      size_t lds_bytes = 0;
      bool in_lds = false;
      if (c.size() == 1) {
        (void)fused_levels<T>(*G, l0, lds_bytes, in_lds);
        ensure_fused_desc<T>(pb, *G, l0);
        launch_vcycle_bottom<T>((const FusedLevels<T>*)G->fdesc, lds_bytes,
                                G->n_list, mask_of(G), sample_list(*G), st);
        continue;
      }
      FusedLevels<T> F = fused_levels<T>(*G, l0, lds_bytes, in_lds);
      F.nu1 = nu1;
      F.nu2 = nu2;
      for (int k = 0; k < F.n; ++k) {
        const Level& X = G->lv[l0 + k];
        const size_t Np = X.g.off[8];
        F.A[k] = (const T*)pool_base(F.A[k], X.slot, kPlanes * Np * tsz);
        F.D[k] = (const T*)pool_base(F.D[k], X.slot, 4 * Np * tsz);
        F.LF[k] = (const T*)pool_base(F.LF[k], X.slot, kLineFactors * Np * tsz);
        F.r[k] = (T*)pool_base(F.r[k], X.slot, 2 * Np * tsz);
        F.b[k] = (T*)pool_base(F.b[k], X.slot, 2 * Np * tsz);
        F.x[k] = (T*)pool_base(F.x[k], X.slot, 2 * Np * tsz);
      }
      F.Minv = (const double*)pool_base(F.Minv, G->lv[G->L - 1].slot,
                                        (size_t)G->n_coarse * G->n_coarse * sizeof(double));
      std::vector<long> key = {F.n, F.nc, F.nu1, F.nu2, F.line_lds, (long)(intptr_t)F.Minv};
      for (int k = 0; k < F.n; ++k)
        for (long v : {(long)F.lds_off[k], (long)F.g[k].nx, (long)F.g[k].ny, (long)F.g[k].nz,
                       (long)(intptr_t)F.A[k], (long)(intptr_t)F.D[k], (long)(intptr_t)F.LF[k],
                       (long)(intptr_t)F.x[k],
                       (long)(intptr_t)F.b[k], (long)(intptr_t)F.r[k]})
          key.push_back(v);
      void* desc = nullptr;
      for (auto& d : pb->mg_bottoms)
        if (d.key == key) desc = d.d;
      if (!desc) {
        char* q = nullptr;
        if (dalloc(pb, &q, sizeof(F))) return;
        (void)hipMemcpyAsync(q, &F, sizeof(F), hipMemcpyHostToDevice, st);
        (void)hipStreamSynchronize(st);
        pb->mg_bottoms.push_back({key, q});
        desc = q;
      }
      std::vector<std::pair<Group*, int>> parts;
      for (Group* H : c) parts.push_back({H, l0of(H)});
      int rows = 0;
      const int* list = merged_list(pb, parts, rows, st);
      launch_vcycle_bottom<T>((const FusedLevels<T>*)desc, lds_bytes, rows,
                              nullptr, list, st);
    }
  }
  for (size_t q = stations.size(); q-- > 0;)
    for (const Target& t : plan[q]) {
      launch_prolong<T>(t.L->g, t.Lc->g, t.xc, t.x, t.rows, t.mask, t.list, st);
      const int ncol = t.ln ? 4 : 8;
      for (int it = 0; it < nu2; ++it)
        for (int c = ncol - 1; c >= 0; --c) smooth(t, c, t.b, t.x, false);
    }
  for (MergeReq* r : W) {
    Group& G = *r->G;
    launch_from_colour<T>(G.lv[0].g, (const T*)G.lv[0].x, r->out, G.n_list, r->mask,
                          sample_list(G), st);
  }
  if (ve1) (void)hipEventRecord(ve1, st);
}

// with every group inside BiCGStab waiting (mg_mu held): their V-cycles in one pass
void merged_run(edf_problem* pb) {
  std::vector<MergeReq*> R;
  R.swap(pb->mg_wait);
  if (mixed(pb))
    vcycle_merged<float>(pb, R);
  else
    vcycle_merged<double>(pb, R);
  for (MergeReq* r : R) r->done = true;
  pb->mg_cv.notify_all();
}

void krylov_enter(edf_problem* pb, Group& G) {
  if (pb->opts.concurrent_groups != 2) return;
  std::lock_guard<std::mutex> lk(pb->mg_mu);
  ++pb->mg_in;
  G.in_krylov = true;
}

void krylov_leave(edf_problem* pb, Group& G) {
  if (!G.in_krylov) return;
  std::lock_guard<std::mutex> lk(pb->mg_mu);
  --pb->mg_in;
  G.in_krylov = false;
  if (!pb->mg_wait.empty() && (int)pb->mg_wait.size() >= pb->mg_in) merged_run(pb);
}

void precondition(edf_problem* pb, Group& G, const double* in, double* out, const int* mask) {
  if (G.in_krylov) {  // wait for the other groups inside BiCGStab, or run all their cycles
    MergeReq r{&G, in, out, mask};
    std::unique_lock<std::mutex> lk(pb->mg_mu);
    pb->mg_wait.push_back(&r);
    if ((int)pb->mg_wait.size() >= pb->mg_in)
      merged_run(pb);
    else
      pb->mg_cv.wait(lk, [&] { return r.done; });
    return;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t tsz = mixed(pb) ? sizeof(float) : sizeof(double);
  const double bytes =
      vcycle_bytes(G, tsz, pb->opts.nu_pre, pb->opts.nu_post, first_fused_level(G)) * G.n_active;
  // captured V-cycles when asked for and not profiling (the profile times single launches)
  if (pb->opts.graph_vcycle && !G.prof_on && G.n_list > 0) {
    if (mixed(pb) ? vcycle_graph<float>(pb, G, in, out, mask)
                  : vcycle_graph<double>(pb, G, in, out, mask))
      return;
  }
  if (prof_pair(G, e0, e1, bytes, 1)) (void)hipEventRecord(e0, G.st);
  if (mixed(pb))
    vcycle<float>(pb, G, in, out, mask);
  else
    vcycle<double>(pb, G, in, out, mask);
  if (e1) (void)hipEventRecord(e1, G.st);
}

// ---------------------------------------------------------------------------
// BiCGStab on A x = F~ for the samples in G.nmask; x in G.kx
// ---------------------------------------------------------------------------
edf_status bicgstab(edf_problem* pb, Group& G) {
  krylov_enter(pb, G);
  struct Leave {
    edf_problem* pb;
    Group& G;
    ~Leave() { krylov_leave(pb, G); }
  } leave{pb, G};
  hipStream_t st = G.st;
  const int S = G.S;
  const size_t n = G.n;
  const Geom& g0 = G.lv[0].g;
  // the products with the assembled stencil, or matrix-free at the current iterate (the
  // adjoint's transposed systems are always assembled)
  JacOp A;
  if (pb->opts.matrix_free && !G.transposed) {
    A.ph = G.lv[0].ph;
    A.dts = G.dts;
    A.phi = G.lv[0].phi;
    A.K = G.lv[0].K;
    A.u = G.u;
  } else {
    A.A = G.lv[0].A64;
  }
  launch_bicg_init(n, G.F, G.kx, G.kr, G.krh, G.kp, G.kv, G.part, G.ks, G.eta, G.active, S,
                   G.nmask, st);
  auto count_active = [&]() -> edf_status {
    EDF_CHECK_LAUNCH();
    EDF_TRY(hipMemcpyAsync(G.h_int, G.active, S * sizeof(int), hipMemcpyDeviceToHost, st));
    EDF_TRY(hipStreamSynchronize(st));
    G.n_active = 0;
    for (int s = 0; s < S; ++s) G.n_active += G.h_int[s] != 0;
    edf_status e;
    if ((e = set_sample_list(pb, G, G.h_int))) return e;
    return prof_flush(pb, G);
  };
  edf_status e;
  if ((e = count_active())) return e;
  const int chunk = std::max(1, pb->opts.check_every);
  for (int it = 0; it < pb->opts.lin_max_it && G.n_active > 0; it += chunk) {
    for (int c = 0; c < chunk && it + c < pb->opts.lin_max_it; ++c) {
      // the launches run over the samples active at the last count (a superset of those
      // still active: the active flags gate the rest)
      const SampleList sl{G.n_list < S ? G.d_list : nullptr, G.n_list};
      launch_bicg_p(n, G.kr, G.kv, G.kp, G.krh, G.ks, S, G.active, sl, st);
      precondition(pb, G, G.kp, G.kph, G.active);
      launch_bicg_alpha(g0, A, G.kph, G.kv, G.krh, G.part, G.ks, S, G.active, sl, st);
      launch_bicg_s(n, G.kr, G.kv, G.ks_, G.part, G.ks, S, G.active, sl, st);
      precondition(pb, G, G.ks_, G.ksh, G.active);
      launch_bicg_omega(g0, A, G.ksh, G.ks_, G.kt, G.part, G.ks, S, G.active, sl, st);
      launch_bicg_update(n, G.kph, G.ksh, G.ks_, G.kt, G.krh, G.kx, G.kr, G.part, G.ks, G.active,
                         S, G.active, sl, st);
    }
    if ((e = count_active())) return e;
  }
  return EDF_OK;
}

edf_status read_norms(edf_problem* pb, Group& G, const double* F, const int* mask,
                      std::vector<double>& out) {
  launch_sq_norm(G.n, F, G.part, G.norms, G.S, mask, G.st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(G.h_dbl, G.norms, G.S * sizeof(double), hipMemcpyDeviceToHost, G.st));
  EDF_TRY(hipStreamSynchronize(G.st));
  out.resize(G.S);
  for (int s = 0; s < G.S; ++s) out[s] = std::sqrt(G.h_dbl[s]);
  return EDF_OK;
}

edf_status upload_ints(edf_problem* pb, Group& G, int* dst, const std::vector<int>& v) {
  EDF_TRY(hipStreamSynchronize(G.st));  // the staging buffer may still feed a copy
  std::copy(v.begin(), v.end(), G.h_int);
  EDF_TRY(hipMemcpyAsync(dst, G.h_int, v.size() * sizeof(int), hipMemcpyHostToDevice, G.st));
  EDF_TRY(hipStreamSynchronize(G.st));
  return EDF_OK;
}

edf_status upload_dbls(edf_problem* pb, Group& G, double* dst, const std::vector<double>& v) {
  EDF_TRY(hipStreamSynchronize(G.st));
  std::copy(v.begin(), v.end(), G.h_dbl);
  EDF_TRY(hipMemcpyAsync(dst, G.h_dbl, v.size() * sizeof(double), hipMemcpyHostToDevice,
                         G.st));
  EDF_TRY(hipStreamSynchronize(G.st));
  return EDF_OK;
}

void set_dt(edf_problem* pb, Group& G, double dt) {
  for (Level& L : G.lv) L.ph = make_phys(pb->phys, L.g, dt);
}

// ---------------------------------------------------------------------------
// autotuning of the fused V-cycle bottom: with the matrices of the current state,
// time three V-cycles for every candidate first fused level and keep the fastest
// ---------------------------------------------------------------------------
edf_status autotune_group(edf_problem* pb, Group& G, bool fuse, bool tiles) {
  hipStream_t st = G.st;
  std::vector<int> all(G.S, 1);
  edf_status e;
  if ((e = upload_ints(pb, G, G.nmask, all))) return e;
  if ((e = set_sample_list(pb, G, all.data()))) return e;
  if ((e = assemble_all(pb, G, G.nmask, nullptr))) return e;
  launch_defect(G.lv[0].g, G.lv[0].ph, nullptr, G.lv[0].phi, G.lv[0].K, G.u, G.u, G.kp, G.S,
                nullptr, st);
  hipEvent_t a, b;
  EDF_TRY(hipEventCreate(&a));
  EDF_TRY(hipEventCreate(&b));
  const bool was_on = G.prof_on;
  G.prof_on = false;
  G.n_active = G.S;
  if (fuse) G.tune_ms.assign(G.L, -1.0);
  // two passes over the candidates, each timing three V-cycles after a warm-up one; a
  // candidate's time is the smaller of its two, so that a slow first pass (caches,
  // clocks) does not decide
  for (int pass = 0; pass < 2 && fuse; ++pass)
    for (int l0 = first_fusable(G); l0 < G.L; ++l0) {
      G.fuse_from = l0;
      precondition(pb, G, G.kp, G.kph, G.nmask);  // warm-up
      EDF_TRY(hipEventRecord(a, st));
      for (int r = 0; r < 3; ++r) precondition(pb, G, G.kp, G.kph, G.nmask);
      EDF_TRY(hipEventRecord(b, st));
      EDF_TRY(hipEventSynchronize(b));
      float ms = 0.f;
      EDF_TRY(hipEventElapsedTime(&ms, a, b));
      if (G.tune_ms[l0] < 0 || ms / 3.0 < G.tune_ms[l0]) G.tune_ms[l0] = ms / 3.0;
    }
  int best_l0 = G.L - 1;
  if (fuse) {
    for (int l0 = first_fusable(G); l0 < G.L; ++l0)
      if (G.tune_ms[l0] < G.tune_ms[best_l0]) best_l0 = l0;
    G.fuse_from = best_l0;
  } else {
    best_l0 = first_fused_level(G);
  }
  // tile shape of the line sweep on every level swept by its own launches, finest first
  // (coordinate descent: the other levels keep their current choice); each candidate's
  // time is the better of two timings of three V-cycles
  const bool mx = mixed(pb);
  for (int l = 0; l < best_l0 && tiles; ++l) {
    Level& L = G.lv[l];
    if (!L.LF) continue;
    double best = -1.0;
    int best_c = L.line_cols;
    for (int c : {8, 16, 32}) {
      if (!(mx ? line_cols_valid<float>(L.g, c) : line_cols_valid<double>(L.g, c))) continue;
      L.line_cols = c;
      for (int pass = 0; pass < 2; ++pass) {
        precondition(pb, G, G.kp, G.kph, G.nmask);
        EDF_TRY(hipEventRecord(a, st));
        for (int r = 0; r < 3; ++r) precondition(pb, G, G.kp, G.kph, G.nmask);
        EDF_TRY(hipEventRecord(b, st));
        EDF_TRY(hipEventSynchronize(b));
        float ms = 0.f;
        EDF_TRY(hipEventElapsedTime(&ms, a, b));
        if (best < 0 || ms / 3.0 < best) {
          best = ms / 3.0;
          best_c = c;
        }
      }
    }
    L.line_cols = best_c;
  }
  G.prof_on = was_on;
  EDF_TRY(hipEventDestroy(a));
  EDF_TRY(hipEventDestroy(b));
  EDF_CHECK_LAUNCH();
  return EDF_OK;
}


// ---------------------------------------------------------------------------
// Newton with line search (Section 2.3) for the samples in `run`, each with its
// own step length in G.dts and previous state in G.u_old.  ok[s] = 1 when the
// sample converged to an admissible state (0 <= c <= 1 up to kRangeTol).
// ---------------------------------------------------------------------------
constexpr double kRangeTol = 0.05;      // admissible overshoot of c beyond [0, 1]
constexpr double kEtaMax = 0.5;         // largest Eisenstat-Walker forcing term
constexpr double kDivergence = 1e4;     // give up when ||F~|| grows by this factor
constexpr int kSlowIts = 8;             // give up after this many iterations ...
constexpr double kSlowDrop = 1e-2;      // ... without this reduction of ||F~||

edf_status newton_solve(edf_problem* pb, Group& G, const std::vector<int>& run,
                        const std::vector<int>& can_retry, std::vector<int>& ok,
                        std::vector<int>& why, bool first_attempt,
                        const std::vector<int>* extrapolate = nullptr) {
  hipStream_t st = G.st;
  const int S = G.S;
  const edf_solver_opts& o = pb->opts;
  const Level& L0 = G.lv[0];
  const double pu = p_unit(pb->phys);
  edf_status e;
  if ((e = upload_ints(pb, G, G.nmask, run))) return e;
  launch_defect(L0.g, L0.ph, G.dts, L0.phi, L0.K, G.u, G.u_old, G.F, S, G.nmask, st);
  std::vector<double> r, r0, rt;
  if ((e = read_norms(pb, G, G.F, G.nmask, r))) return e;
  r0 = r;
  std::vector<int> nm(run), ls(S), acc(S);
  // extrapolated start (opts.predictor) for the samples flagged in `extrapolate`: Newton
  // starts from 2 u^n - u^{n-1} where its scaled defect is below that of u^n; r0 stays the
  // defect at u^n, so the stopping test asks for the same accuracy
  if (extrapolate) {
    bool any_x = false;
    for (int s = 0; s < S; ++s) {
      ls[s] = run[s] && (*extrapolate)[s] && std::isfinite(r[s]);
      any_x |= ls[s] != 0;
    }
    if (any_x) {
      if ((e = upload_ints(pb, G, G.lsmask, ls))) return e;
      launch_extrapolate(G.n, G.u, G.u_prev, G.ut, S, G.lsmask, st);
      launch_defect(L0.g, L0.ph, G.dts, L0.phi, L0.K, G.ut, G.u_old, G.Ft, S, G.lsmask, st);
      std::vector<double> rx;
      if ((e = read_norms(pb, G, G.Ft, G.lsmask, rx))) return e;
      for (int s = 0; s < S; ++s) {
        acc[s] = ls[s] && rx[s] < r[s];
        if (acc[s]) r[s] = rx[s];
        if (first_attempt && run[s]) G.stats[s].predicted = acc[s];
      }
      if ((e = upload_ints(pb, G, G.lsmask, acc))) return e;
      launch_masked_copy(G.n, G.ut, G.u, S, G.lsmask, st);
      launch_masked_copy(G.n, G.Ft, G.F, S, G.lsmask, st);
    }
  }
  std::vector<double> lam(S), eta(S, o.lin_rtol), r_prev(S, 0.0);
  ok.assign(S, 0);
  why.assign(S, EDF_SAMPLE_OK);
  for (int s = 0; s < S; ++s) {
    if (!run[s]) continue;
    if (first_attempt) G.stats[s].defect0 = r0[s];
    G.stats[s].defect = r[s];
    if (!std::isfinite(r0[s])) {
      why[s] = EDF_SAMPLE_NONFINITE;
      nm[s] = 0;
    }
  }
  for (int it = 0;; ++it) {
    bool any = false;
    for (int s = 0; s < S; ++s) {
      if (!nm[s]) continue;
      if (r[s] <= std::max(o.newton_rtol * r0[s], o.newton_atol)) {
        nm[s] = 0;
        ok[s] = 1;
      } else if (it >= o.newton_max_it || (it >= kSlowIts && r[s] > kSlowDrop * r0[s])) {
        nm[s] = 0;
        why[s] = EDF_SAMPLE_NEWTON_FAIL;
      } else {
        any = true;
      }
    }
    if (!any) break;
    // relative tolerance of this Newton system: fixed, or the Eisenstat-Walker forcing
    // term (choice 2: 0.9 (r_k / r_{k-1})^2, safeguarded, at most kEtaMax), never asking
    // for more than half of what is left to the Newton target
    for (int s = 0; s < S; ++s) {
      if (!nm[s] || o.forcing == 0) continue;
      double et = kEtaMax;
      if (it > 0) {
        const double q = r[s] / r_prev[s];
        et = 0.9 * q * q;
        const double prev = 0.9 * eta[s] * eta[s];
        if (prev > 0.1) et = std::max(et, prev);
      }
      et = std::min(et, kEtaMax);
      const double target = std::max(o.newton_rtol * r0[s], o.newton_atol);
      et = std::max(et, 0.5 * target / r[s]);
      eta[s] = std::max(std::min(et, kEtaMax), o.lin_rtol);
    }
    for (int s = 0; s < S; ++s) r_prev[s] = r[s];
    if ((e = upload_dbls(pb, G, G.eta, eta))) return e;
    if ((e = upload_ints(pb, G, G.nmask, nm))) return e;
    if (it == 0 || !o.lag_preconditioner)
      if ((e = assemble_all(pb, G, G.nmask, G.dts))) return e;
    if ((e = bicgstab(pb, G))) return e;
    // BiCGStab statistics and the size of the Newton update
    EDF_TRY(hipMemcpyAsync(G.h_ks, G.ks, S * sizeof(KrylovScalars), hipMemcpyDeviceToHost, st));
    std::vector<double> dnorm;
    if ((e = read_norms(pb, G, G.kx, G.nmask, dnorm))) return e;
    for (int s = 0; s < S; ++s)
      if (nm[s]) {
        G.stats[s].newton_its += 1;
        G.stats[s].lin_its += G.h_ks[s].it;
        // BiCGStab ended more than a factor 2 short of its tolerance: the preconditioner
        // is not up to this time step, and a shorter one is cheaper than inexact Newton
        const KrylovScalars& k = G.h_ks[s];
        if (can_retry[s] && k.state != 1 && !(k.rr <= 4.0 * k.tol2)) {
          nm[s] = 0;
          why[s] = EDF_SAMPLE_LINEAR_FAIL;
        }
      }
    // line search on u - lambda * x  (x solves A x = F~, so the Newton step is -x)
    double l = 1.0;
    for (int s = 0; s < S; ++s) {
      ls[s] = nm[s];
      lam[s] = -1.0;
    }
    rt = r;
    for (int h = 0; h <= o.ls_max_halvings; ++h) {
      bool any_ls = false;
      for (int s = 0; s < S; ++s) any_ls |= ls[s] != 0;
      if (!any_ls) break;
      if ((e = upload_ints(pb, G, G.lsmask, ls))) return e;
      if ((e = upload_dbls(pb, G, G.lam, lam))) return e;
      launch_axpy_state(G.N, G.u, G.kx, G.lam, pu, G.ut, S, G.lsmask, st);
      launch_defect(L0.g, L0.ph, G.dts, L0.phi, L0.K, G.ut, G.u_old, G.Ft, S, G.lsmask, st);
      std::vector<double> rr;
      if ((e = read_norms(pb, G, G.Ft, G.lsmask, rr))) return e;
      for (int s = 0; s < S; ++s) {
        if (!ls[s]) continue;
        rt[s] = rr[s];
        const bool decrease = rr[s] <= (1.0 - l / 4.0) * r[s];
        if (decrease || h == o.ls_max_halvings) {
          ls[s] = 0;
        } else {
          lam[s] *= 0.5;
          G.stats[s].ls_halvings += 1;
        }
      }
      l *= 0.5;
    }
    // accept the trial states that are finite; a non-finite trial ends the attempt
    for (int s = 0; s < S; ++s) {
      acc[s] = 0;
      if (!nm[s]) continue;
      if (!std::isfinite(rt[s]) || rt[s] > kDivergence * r0[s]) {
        nm[s] = 0;
        why[s] = std::isfinite(rt[s]) ? EDF_SAMPLE_NEWTON_FAIL : EDF_SAMPLE_NONFINITE;
        continue;
      }
      acc[s] = 1;
    }
    if ((e = upload_ints(pb, G, G.lsmask, acc))) return e;
    launch_masked_copy(G.n, G.ut, G.u, S, G.lsmask, st);
    launch_masked_copy(G.n, G.Ft, G.F, S, G.lsmask, st);
    for (int s = 0; s < S; ++s)
      if (acc[s]) {
        r[s] = rt[s];
        G.stats[s].defect = rt[s];
        if (std::fabs(lam[s]) * dnorm[s] <= kUpdateFloor * std::sqrt((double)G.n)) {
          nm[s] = 0;  // the update is at the rounding level of the scaled unknowns: converged
          ok[s] = 1;
        }
      }
  }
  // admissibility of the converged states: the salt mass fraction stays in [0, 1]
  bool any_ok = false;
  for (int s = 0; s < S; ++s) any_ok |= ok[s] != 0;
  if (any_ok) {
    if ((e = upload_ints(pb, G, G.lsmask, ok))) return e;
    launch_c_range(L0.g, G.u, G.part, G.crange, S, G.lsmask, st);
    EDF_CHECK_LAUNCH();
    std::vector<double> cr(2 * S);
    EDF_TRY(hipMemcpyAsync(cr.data(), G.crange, 2 * S * sizeof(double), hipMemcpyDeviceToHost, st));
    EDF_TRY(hipStreamSynchronize(st));
    for (int s = 0; s < S; ++s)
      if (ok[s] && !(cr[2 * s] >= -kRangeTol && cr[2 * s + 1] <= 1.0 + kRangeTol)) {
        ok[s] = 0;
        why[s] = EDF_SAMPLE_INADMISSIBLE;
      }
  }
  EDF_CHECK_LAUNCH();
  return EDF_OK;
}

// ---------------------------------------------------------------------------
// one time step of length DT for every sample of a group that has not failed.  A
// sample whose Newton solve fails restarts the step from its saved state as 2^h equal
// sub-steps of DT / 2^h (h <= dt_max_halvings); samples advance in lockstep, one
// sub-step each per round, and finished samples are masked out.  After every sub-step
// that converged, the FP64 mass balance of that sub-step is added up on the device.
// ---------------------------------------------------------------------------
edf_status macro_step(edf_problem* pb, Group& G, double DT) {
  hipStream_t st = G.st;
  const int S = G.S;
  set_dt(pb, G, DT);
  edf_status e;
  EDF_TRY(hipMemcpyAsync(G.u0, G.u, S * G.n * sizeof(double), hipMemcpyDeviceToDevice, st));
  const bool memory = pb->opts.substep_memory != 0;
  if ((int)G.h_start.size() != S) reset_history(G);
  std::vector<int> h(S, 0), done(S, 0), running(S, 0), started(S, 0), ok, why, restore(S),
      can_retry(S);
  std::vector<double> dts(S);
  for (int s = 0; s < S; ++s) {
    edf_step_stats& t = G.stats[s];
    t.status = G.fail_status[s];
    t.newton_its = t.lin_its = t.ls_halvings = t.retries = 0;
    t.substeps = 0;
    t.predicted = 0;
    t.defect0 = t.defect = 0.0;
    t.salt_balance_err = t.liquid_balance_err = 0.0;
    if (G.fail_status[s] != EDF_SAMPLE_OK) continue;  // failed in an earlier step
    running[s] = started[s] = 1;
    h[s] = memory ? std::min(G.h_start[s], pb->opts.dt_max_halvings) : 0;
    t.substeps = 1 << h[s];
  }
  launch_fill<double>(G.bal, 8, S, nullptr, 0.0, st);
  const Level& L0 = G.lv[0];
  bool first = true;
  // extrapolated Newton starts (opts.predictor): the samples whose previous step was one
  // implicit-Euler step of this length and that try the full length now
  std::vector<int> extrap(S, 0);
  const bool predict = G.u_prev && !pb->recording;
  if (predict)
    for (int s = 0; s < S; ++s) extrap[s] = running[s] && h[s] == 0 && G.pred_dt[s] == DT;
  for (;;) {
    bool any = false;
    for (int s = 0; s < S; ++s) {
      any |= running[s] != 0;
      dts[s] = DT / double(1 << h[s]);
    }
    if (!any) break;
    if ((e = upload_dbls(pb, G, G.dts, dts))) return e;
    if ((e = upload_ints(pb, G, G.nmask, running))) return e;
    launch_masked_copy(G.n, G.u, G.u_old, S, G.nmask, st);
    for (int s = 0; s < S; ++s) can_retry[s] = h[s] < pb->opts.dt_max_halvings;
    if ((e = newton_solve(pb, G, running, can_retry, ok, why, first,
                          first && predict ? &extrap : nullptr)))
      return e;
    first = false;
    // mass balance of the sub-steps that converged (u: their end, u_old: their start)
    bool any_ok = false;
    for (int s = 0; s < S; ++s) any_ok |= running[s] && ok[s];
    if (any_ok) {
      if ((e = upload_ints(pb, G, G.lsmask, ok))) return e;
      launch_balance(L0.g, L0.ph, G.dts, L0.phi, L0.K, G.u, G.u_old, G.bal_part, G.bal, S,
                     G.lsmask, st);
    }
    bool any_restore = false;
    for (int s = 0; s < S; ++s) {
      restore[s] = 0;
      if (!running[s]) continue;
      if (ok[s]) {
        if (++done[s] == (1 << h[s])) running[s] = 0;
        continue;
      }
      restore[s] = 1;
      any_restore = true;
      done[s] = 0;
      if (h[s] < pb->opts.dt_max_halvings) {
        h[s] += 1;
        G.stats[s].substeps = 1 << h[s];
        G.stats[s].retries += 1;
      } else {
        running[s] = 0;
        G.stats[s].status = why[s];
      }
    }
    if (any_restore) {
      if ((e = upload_ints(pb, G, G.lsmask, restore))) return e;
      launch_masked_copy(G.n, G.u0, G.u, S, G.lsmask, st);
      launch_fill<double>(G.bal, 8, S, G.lsmask, 0.0, st);  // the balance starts again too
    }
  }
  EDF_CHECK_LAUNCH();
  std::vector<double> bal(8 * (size_t)S);
  EDF_TRY(hipMemcpyAsync(bal.data(), G.bal, bal.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipStreamSynchronize(st));
  for (int s = 0; s < S; ++s) {
    if (!started[s]) continue;
    edf_step_stats& t = G.stats[s];
    t.retries_total += t.retries;
    if (t.status != EDF_SAMPLE_OK) {  // failed: keeps its state from the start of the step
      G.fail_status[s] = t.status;
      t.failed_step = t.steps_total + 1;
      continue;
    }
    t.steps_total += 1;
    t.substeps_total += t.substeps;
    t.split_total += t.substeps > 1;
    // |dM - B| relative to the mass moved (the storage changes' absolute sum and B)
    const double* b = &bal[8 * (size_t)s];
    auto rel = [](double dM, double gross, double B) {
      const double den = gross + std::fabs(B);
      return den > 0.0 ? std::fabs(dM - B) / den : 0.0;
    };
    t.salt_balance_err = rel(b[0], b[1], b[4]);
    t.liquid_balance_err = rel(b[2], b[3], b[5]);
  }
  // history of the extrapolated start: this step's start state for the samples that took
  // it as one implicit-Euler step
  if (G.u_prev) {
    std::vector<int> keep(S, 0);
    for (int s = 0; s < S; ++s) {
      keep[s] = started[s] && G.stats[s].status == EDF_SAMPLE_OK && G.stats[s].substeps == 1;
      G.pred_dt[s] = keep[s] ? DT : 0.0;
    }
    if ((e = upload_ints(pb, G, G.lsmask, keep))) return e;
    launch_masked_copy(G.n, G.u0, G.u_prev, S, G.lsmask, st);
  }
  // the next step starts with the sub-step count that worked; after `wait` steps
  // without a retry it tries one halving less, and every such try that fails
  // doubles `wait` (3 at first, at most kMaxWait)
  if (memory)
    for (int s = 0; s < S; ++s) {
      if (!started[s] || G.stats[s].status != EDF_SAMPLE_OK) continue;
      if (h[s] == G.h_start[s]) {
        if (G.probing[s]) G.wait[s] = kFirstWait;
        G.probing[s] = 0;
        if (++G.clean[s] >= G.wait[s] && h[s] > 0) {
          G.h_start[s] = h[s] - 1;
          G.clean[s] = 0;
          G.probing[s] = 1;
        }
      } else {
        if (G.probing[s]) G.wait[s] = std::min(2 * G.wait[s], kMaxWait);
        G.probing[s] = 0;
        G.h_start[s] = h[s];
        G.clean[s] = 0;
      }
    }
  return EDF_OK;
}

// ---------------------------------------------------------------------------
// adjoint: matrices of every level transposed, at the current iterate
// ---------------------------------------------------------------------------
edf_status assemble_all_transposed(edf_problem* pb, Group& G, const int* mask, const double* dts) {
  const bool mx = mixed(pb);
  G.transposed = true;
  for (int l = 0; l < G.L; ++l) {
    Level& L = G.lv[l];
    if (l > 0) launch_inject(G.lv[l - 1].g, L.g, G.lv[l - 1].u, L.u, G.S, mask, G.st);
    const bool coarsest = l == G.L - 1;
    if (l == 0) {  // exact Jacobian, transposed, for the Krylov products
      launch_assemble(L.g, L.ph, dts, L.phi, L.K, L.u, G.tmpA, nullptr, G.S, mask, G.st, false);
      launch_transpose<double>(L.g, G.tmpA, L.A64, G.S, mask, G.st);
    }
    launch_assemble(L.g, L.ph, dts, L.phi, L.K, L.u, G.tmpA, nullptr, G.S, mask, G.st, true);
    if (mx && !coarsest) {
      launch_transpose<float>(L.g, G.tmpA, L.A32, G.S, mask, G.st);
      if (l == 0 && f16_finest(pb, G))
        launch_scale_f16(L.g, L.A32, L.A16, (float*)L.Dinv, G.S, mask, G.st);
      else
        launch_block_inverse_f32(L.g, L.A32, (float*)L.Dinv, G.S, mask, G.st);
    } else {
      double* m64 = l == 0 ? L.AV64 : L.A64;
      launch_transpose<double>(L.g, G.tmpA, m64, G.S, mask, G.st);
      if (!coarsest) launch_block_inverse_f64(L.g, m64, (double*)L.Dinv, G.S, mask, G.st);
    }
    if (!coarsest) line_factors(L, mx, G.S, mask, G.st);
  }
  const Level& C = G.lv[G.L - 1];
  launch_coarse_dense(C.g, G.L == 1 ? C.AV64 : C.A64, G.Minv, G.S, mask, G.st);
  launch_gauss_jordan(G.n_coarse, G.Minv, G.piv, G.gj_status, G.S, mask, G.st);
  EDF_CHECK_LAUNCH();
  return EDF_OK;
}

// buffers of a recorded trajectory of n_steps steps with a checkpoint every k steps
edf_status ensure_trajectory_buffers(edf_problem* pb, Group& G, int n_steps, int k) {
  const size_t S = G.S, n = G.n;
  edf_status e;
  const size_t nck = (size_t)ceil_div(n_steps, k) + 1;
  if (G.ckpt_cap < nck) {
    if (G.ckpt) (void)hipFree(G.ckpt);
    G.ckpt = nullptr;
    G.ckpt_cap = 0;
    EDF_TRY(hipMalloc((void**)&G.ckpt, S * nck * n * sizeof(double)));
    G.ckpt_cap = nck;
  }
  if (!G.idx && (e = dalloc(pb, &G.idx, S))) return e;  // slot indices of gather/scatter
  return EDF_OK;
}

// buffers of the backward sweep: one segment of k + 1 states, the sub-step states of one
// step, the adjoint state and the transposition scratch
edf_status ensure_adjoint_buffers(edf_problem* pb, Group& G, int k) {
  const size_t S = G.S, n = G.n;
  edf_status e;
  if (G.seg_cap < (size_t)k + 1) {
    if (G.seg) (void)hipFree(G.seg);
    G.seg = nullptr;
    G.seg_cap = 0;
    EDF_TRY(hipMalloc((void**)&G.seg, S * ((size_t)k + 1) * n * sizeof(double)));
    G.seg_cap = (size_t)k + 1;
  }
  const size_t kmax = (size_t(1) << pb->opts.dt_max_halvings) + 1;
  if (G.sub_cap < kmax) {
    G.sub_cap = kmax;
    if ((e = dalloc(pb, &G.sub, S * G.sub_cap * n))) return e;
  }
  if (!G.lv[0].A64 && (e = dalloc(pb, &G.lv[0].A64, S * kPlanes * (size_t)G.lv[0].g.off[8])))
    return e;  // the transposed exact Jacobian (assembled also with matrix-free forward products)
  if (!G.lam_next) {
    if ((e = dalloc(pb, &G.lam_next, S * n))) return e;
    if ((e = dalloc(pb, &G.tmpA, S * kPlanes * (size_t)G.lv[0].g.off[8]))) return e;
    if ((e = dalloc(pb, &G.g4, 4 * S))) return e;
  }
  return EDF_OK;
}

// d = state slot idx[s] of buf ([S][cap][n]) for every sample with idx[s] >= 0
edf_status gather(edf_problem* pb, Group& G, const double* buf, size_t cap,
                  const std::vector<int>& idx, double* dst) {
  edf_status e;
  if ((e = upload_ints(pb, G, G.idx, idx))) return e;
  launch_gather_state(G.n, buf, cap * G.n, G.idx, dst, G.S, G.st);
  return EDF_OK;
}

edf_status scatter(edf_problem* pb, Group& G, const double* src, double* buf, size_t cap,
                   const std::vector<int>& idx) {
  edf_status e;
  if ((e = upload_ints(pb, G, G.idx, idx))) return e;
  launch_scatter_state(G.n, src, buf, cap * G.n, G.idx, G.S, G.st);
  return EDF_OK;
}

// Replays sub-steps of one recorded step from the states in G.u: sample s takes its
// sub-steps r = 1 .. r_end[s] of length dt / K[s] (K[s] = 0: left alone).  When to_sub,
// the state after sub-step r is stored in slot r of G.sub.  The forward attempt at this
// sub-step length converged, so no Krylov failure ended it: replaying without that check
// takes the same path, and the deterministic kernels give the same states bitwise.
edf_status replay_substeps(edf_problem* pb, Group& G, double dt, const std::vector<int>& K,
                           const std::vector<int>& r_end, bool to_sub) {
  const int S = G.S;
  edf_status e;
  std::vector<double> dts(S, dt);
  std::vector<int> act(S), okv, why, idx(S);
  int rmax = 0;
  for (int s = 0; s < S; ++s) {
    if (K[s] > 0) dts[s] = dt / K[s];
    rmax = std::max(rmax, r_end[s]);
  }
  if (rmax == 0) return EDF_OK;
  set_dt(pb, G, dt);
  if ((e = upload_dbls(pb, G, G.dts, dts))) return e;
  for (int r = 1; r <= rmax; ++r) {
    for (int s = 0; s < S; ++s) act[s] = K[s] > 0 && r <= r_end[s];
    if ((e = upload_ints(pb, G, G.nmask, act))) return e;
    launch_masked_copy(G.n, G.u, G.u_old, S, G.nmask, G.st);
    if ((e = newton_solve(pb, G, act, std::vector<int>(S, 0), okv, why, false))) return e;
    for (int s = 0; s < S; ++s)
      if (act[s] && !okv[s])
        return fail(pb, EDF_ERR_STATE, "recomputation of a recorded sub-step failed for sample " +
                                           std::to_string(G.s0 + s));
    if (to_sub) {
      for (int s = 0; s < S; ++s) idx[s] = act[s] ? r : -1;
      if ((e = scatter(pb, G, G.u, G.sub, G.sub_cap, idx))) return e;
    }
  }
  return EDF_OK;
}

// default relative tolerance of the adjoint solves (the gradient amplifies their residual)
constexpr double kAdjointRtol = 1e-12;

// The backward sweep over the trajectory recorded by edf_solve (n steps of dt, a
// checkpoint every k steps): segments from the last, each recomputed from its checkpoint
// into G.seg, then its steps backwards, each through its sub-steps.  J[s] and dJ[s][4]
// of the group's samples (NaN for samples that failed while the trajectory was recorded).
edf_status adjoint_group(edf_problem* pb, Group& G, const QoiBox& box, double rtol,
                         std::vector<double>& Jv, std::vector<double>& grad) {
  hipStream_t st = G.st;
  const int S = G.S;
  const int k = pb->traj_k, n_steps = pb->traj_n;
  const double dt = pb->traj_dt;
  edf_status e;
  if ((e = ensure_adjoint_buffers(pb, G, k))) return e;
  const Level& L0 = G.lv[0];
  FieldParams fp{pb->phys.lx, pb->phys.ly, pb->phys.lz, pb->phys.phi_mean, pb->phys.K_mean,
                 pb->phys.field_model, pb->phys.n_xi};
  const double* dxi = pb->dxi + (size_t)G.s0 * std::max(pb->phys.n_xi, 1);
  Jv.assign(S, 0.0);
  grad.assign(4 * (size_t)S, 0.0);
  std::vector<double> hg(4 * S), eta(S, rtol);
  std::vector<int> K(S), act(S), idx(S), full(S);
  const int n_seg = ceil_div(n_steps, k);
  const int last_slot = n_seg;  // the final state (slot of step n_steps)
  bool first = true;
  for (int sg = n_seg - 1; sg >= 0; --sg) {
    const int a = sg * k, b = std::min(n_steps, a + k);
    // the segment's states: slot 0 from the checkpoint, slots 1 .. b-a-1 recomputed
    // step by step, slot b-a from the next checkpoint (or the final state)
    for (int s = 0; s < S; ++s) idx[s] = G.traj_fail[s] ? -1 : sg;
    if ((e = gather(pb, G, G.ckpt, G.ckpt_cap, idx, G.u))) return e;
    for (int s = 0; s < S; ++s) idx[s] = G.traj_fail[s] ? -1 : 0;
    if ((e = scatter(pb, G, G.u, G.seg, G.seg_cap, idx))) return e;
    for (int m = a; m + 1 < b; ++m) {
      for (int s = 0; s < S; ++s) {
        K[s] = G.traj_fail[s] ? 0 : 1 << G.H[m][s];
        full[s] = K[s];
      }
      if ((e = replay_substeps(pb, G, dt, K, full, false))) return e;
      for (int s = 0; s < S; ++s) idx[s] = G.traj_fail[s] ? -1 : m - a + 1;
      if ((e = scatter(pb, G, G.u, G.seg, G.seg_cap, idx))) return e;
    }
    for (int s = 0; s < S; ++s) idx[s] = G.traj_fail[s] ? -1 : (b == n_steps ? last_slot : sg + 1);
    if ((e = gather(pb, G, G.ckpt, G.ckpt_cap, idx, G.u))) return e;
    for (int s = 0; s < S; ++s) idx[s] = G.traj_fail[s] ? -1 : b - a;
    if ((e = scatter(pb, G, G.u, G.seg, G.seg_cap, idx))) return e;
    for (int m = b - 1; m >= a; --m) {
      int kmax = 0;
      for (int s = 0; s < S; ++s) {
        K[s] = G.traj_fail[s] ? 0 : 1 << G.H[m][s];
        full[s] = std::max(K[s] - 1, 0);
        kmax = std::max(kmax, K[s]);
      }
      // sub-step states of step m: slot 0 = the step's start, slot K = its end, the
      // others recomputed
      for (int s = 0; s < S; ++s) idx[s] = K[s] ? m - a : -1;
      if ((e = gather(pb, G, G.seg, G.seg_cap, idx, G.u))) return e;
      for (int s = 0; s < S; ++s) idx[s] = K[s] ? 0 : -1;
      if ((e = scatter(pb, G, G.u, G.sub, G.sub_cap, idx))) return e;
      if ((e = replay_substeps(pb, G, dt, K, full, true))) return e;
      for (int s = 0; s < S; ++s) idx[s] = K[s] ? m - a + 1 : -1;
      if ((e = gather(pb, G, G.seg, G.seg_cap, idx, G.u))) return e;
      for (int s = 0; s < S; ++s) idx[s] = K[s] ? K[s] : -1;
      if ((e = scatter(pb, G, G.u, G.sub, G.sub_cap, idx))) return e;
      std::vector<double> dts(S, dt);
      for (int s = 0; s < S; ++s)
        if (K[s]) dts[s] = dt / K[s];
      set_dt(pb, G, dt);
      if ((e = upload_dbls(pb, G, G.dts, dts))) return e;
      // backward through the sub-steps, one round per sub-step position
      for (int r = 0; r < kmax; ++r) {
        for (int s = 0; s < S; ++s) {
          act[s] = K[s] > r;
          idx[s] = act[s] ? K[s] - r : -1;
        }
        if ((e = gather(pb, G, G.sub, G.sub_cap, idx, G.u))) return e;
        for (int s = 0; s < S; ++s) idx[s] = act[s] ? K[s] - r - 1 : -1;
        if ((e = gather(pb, G, G.sub, G.sub_cap, idx, G.u_old))) return e;
        if ((e = upload_ints(pb, G, G.nmask, act))) return e;
        if (first) {  // J and dJ/du~ at the final state
          const int nb = ceil_div(L0.g.N, kBlock);
          launch_qoi(L0.g, L0.ph, box, L0.phi, G.u, G.F, G.part, S, G.nmask, st);
          launch_sum4(nb, G.part, G.g4, S, G.nmask, st);
          EDF_CHECK_LAUNCH();
          EDF_TRY(hipMemcpyAsync(hg.data(), G.g4, 4 * S * sizeof(double), hipMemcpyDeviceToHost, st));
          EDF_TRY(hipStreamSynchronize(st));
          for (int s = 0; s < S; ++s) Jv[s] = act[s] ? hg[4 * s] : 0.0;
        } else {
          launch_adjoint_rhs(L0.g, L0.ph, L0.phi, G.u, G.lam_next, G.F, S, G.nmask, st);
        }
        if ((e = assemble_all_transposed(pb, G, G.nmask, G.dts))) return e;
        if ((e = upload_dbls(pb, G, G.eta, eta))) return e;
        if ((e = bicgstab(pb, G))) return e;
        EDF_TRY(hipMemcpyAsync(G.h_ks, G.ks, S * sizeof(KrylovScalars), hipMemcpyDeviceToHost, st));
        EDF_TRY(hipStreamSynchronize(st));
        for (int s = 0; s < S; ++s)
          if (act[s] && G.h_ks[s].state != 1 && G.h_ks[s].bb > 0) {
            const KrylovScalars& k = G.h_ks[s];
            char buf[256];
            std::snprintf(buf, sizeof buf,
                          "adjoint BiCGStab did not converge for sample %d (step %d, %s after %d "
                          "iterations and %d restarts, |r|/|b| = %.3e for a tolerance of %.1e)",
                          G.s0 + s, m, k.state == 2 ? "breakdown" : "iteration limit", k.it,
                          k.restarts, std::sqrt(k.rr / k.bb), std::sqrt(k.tol2 / k.bb));
            return fail(pb, EDF_ERR_NO_CONVERGENCE, buf);
          }
        const int nb = launch_param_grad(L0.g, L0.ph, G.dts, fp, dxi, L0.phi, L0.K, G.u, G.u_old,
                                         G.kx, box, first ? 1 : 0, G.part, S, G.nmask, st);
        launch_sum4(nb, G.part, G.g4, S, G.nmask, st);
        launch_masked_copy(G.n, G.kx, G.lam_next, S, G.nmask, st);
        EDF_CHECK_LAUNCH();
        EDF_TRY(hipMemcpyAsync(hg.data(), G.g4, 4 * S * sizeof(double), hipMemcpyDeviceToHost, st));
        EDF_TRY(hipStreamSynchronize(st));
        for (int s = 0; s < S; ++s)
          if (act[s])
            for (int q = 0; q < 4; ++q) grad[4 * s + q] += hg[4 * s + q];
        first = false;
      }
    }
  }
  for (int s = 0; s < S; ++s)
    if (G.traj_fail[s]) {
      Jv[s] = std::nan("");
      for (int q = 0; q < 4; ++q) grad[4 * s + q] = std::nan("");
    }
  // leave the final states as the problem's states
  for (int s = 0; s < S; ++s) idx[s] = last_slot;
  if ((e = gather(pb, G, G.ckpt, G.ckpt_cap, idx, G.u))) return e;
  EDF_TRY(hipMemcpyAsync(G.u_old, G.u, G.S * G.n * sizeof(double), hipMemcpyDeviceToDevice, st));
  EDF_TRY(hipStreamSynchronize(st));
  return EDF_OK;
}

// ---------------------------------------------------------------------------
// polynomial chaos: the multi-index set J_{M,p} (total degree <= p, or every degree
// <= p), ordered by total degree and then decreasingly lexicographic
// ---------------------------------------------------------------------------
void gpc_indices(int M, int p, int truncation, std::vector<int>& out) {
  out.clear();
  std::vector<int> b(M);
  // all tuples of total t with components <= p, first component largest first
  std::function<void(int, int)> rec = [&](int j, int rem) {
    if (j == M - 1) {
      if (rem <= p) {
        b[j] = rem;
        out.insert(out.end(), b.begin(), b.end());
      }
      return;
    }
    for (int v = std::min(p, rem); v >= 0; --v) {
      b[j] = v;
      rec(j + 1, rem - v);
    }
  };
  const int tmax = truncation == 0 ? p : M * p;
  for (int t = 0; t <= tmax; ++t) rec(0, t);
}

template <typename T>
edf_status grow(edf_problem* pb, T** buf, size_t* cap, size_t need) {
  if (need <= *cap) return EDF_OK;
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *cap = 0;
  EDF_TRY(hipMalloc((void**)buf, need * sizeof(T)));
  *cap = need;
  return EDF_OK;
}

// ---------------------------------------------------------------------------
// Scratch memory of edf_moments_noalloc: a file-scope device array (every device the
// library runs on holds its own copy until the process ends).  Host code never uses the
// array's name as an address: each device's copy is located once, with that device
// current, when the first problem is created on it, and that address is used after.
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = size_t(1) << 21;  // 16 MiB
constexpr int kMaxDevices = 64;
}  // namespace
namespace edf {
// external linkage: the device array must stay in the code object although no kernel
// names it (kernels receive its address as an argument)
__device__ __align__(256) double scratch[kScratchDoubles];
}  // namespace edf
namespace {
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
std::string g_scratch_err[kMaxDevices];

void locate_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device] || !g_scratch_err[device].empty()) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_scratch_err[device] = std::string("hipGetSymbolAddress of the scratch array failed: ") +
                            hipGetErrorString(e);
    return;
  }
  g_scratch[device] = static_cast<double*>(p);
}

edf_status check_ready(edf_problem* pb) {
  if (!pb) return EDF_ERR_ARG;
  if (!pb->params_set) return fail(pb, EDF_ERR_STATE, "edf_set_parameters has not been called");
  return EDF_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

edf_status edf_create_problem(const edf_physics* phys, const edf_group_desc* groups,
                              int32_t n_groups, const edf_solver_opts* opts, void* hip_stream,
                              edf_problem** out) {
  if (!out) return EDF_ERR_ARG;
  *out = nullptr;
  if (!phys || !groups || n_groups <= 0 || !opts) return EDF_ERR_ARG;
  edf_problem* pb = new (std::nothrow) edf_problem();
  if (!pb) return EDF_ERR_OOM;
  pb->phys = *phys;
  pb->opts = *opts;
  pb->st = (hipStream_t)hip_stream;
  if (hipGetDevice(&pb->device) != hipSuccess) {
    delete pb;
    return EDF_ERR_HIP;
  }
  locate_scratch(pb->device);  // once per device (edf_moments_noalloc)
  const edf_physics& P = *phys;
  auto bad = [&](const std::string& m) {
    std::fprintf(stderr, "edf_create_problem: %s\n", m.c_str());
    edf_destroy(pb);
    return EDF_ERR_ARG;
  };
  if (!(P.lx > 0 && P.ly > 0 && P.lz > 0 && P.rho0 > 0 && P.rho1 > 0 && P.mu > 0 && P.g >= 0 &&
        P.Dm >= 0 && P.phi_mean > 0 && P.phi_mean < 1 && P.K_mean > 0))
    return bad("invalid physical constants");
  const int nxi_needed[4] = {0, 1, 4, 3};
  if (P.field_model < 0 || P.field_model > 3 || P.n_xi < nxi_needed[P.field_model] || P.n_xi > 16)
    return bad("invalid field model or n_xi");
  if (opts->precision != EDF_PREC_F64 && opts->precision != EDF_PREC_MIXED &&
      opts->precision != EDF_PREC_MIXED_F16)
    return bad("invalid precision");
  if (opts->newton_max_it < 1 || opts->lin_max_it < 1 || opts->nu_pre < 1 || opts->nu_post < 0 ||
      opts->ls_max_halvings < 0 || !(opts->lin_rtol > 0) || !(opts->newton_rtol >= 0))
    return bad("invalid solver options");
  if (opts->predictor != 0 && opts->predictor != 1) return bad("predictor must be 0 or 1");
  if (opts->lag_preconditioner != 0 && opts->lag_preconditioner != 1)
    return bad("lag_preconditioner must be 0 or 1");
  if (opts->matrix_free != 0 && opts->matrix_free != 1) return bad("matrix_free must be 0 or 1");
  if (opts->graph_vcycle != 0 && opts->graph_vcycle != 1)
    return bad("graph_vcycle must be 0 or 1");
  if (opts->concurrent_groups < 0 || opts->concurrent_groups > 2)
    return bad("concurrent_groups must be 0, 1 or 2");
  if (opts->forcing != 0 && opts->forcing != 1) return bad("forcing must be 0 or 1");
  if (opts->smoother != 0 && opts->smoother != 1) return bad("smoother must be 0 or 1");
  if (opts->substep_memory != 0 && opts->substep_memory != 1)
    return bad("substep_memory must be 0 or 1");
  if (opts->dt_max_halvings < 0 || opts->dt_max_halvings > 12)
    return bad("dt_max_halvings must be in [0, 12]");
  int s0 = 0;
  for (int gi = 0; gi < n_groups; ++gi) {
    const edf_group_desc& d = groups[gi];
    if (d.n_levels < 1 || d.n_levels > 12 || d.n_samples < 1) return bad("invalid group");
    const int r = 1 << (d.n_levels - 1);
    if (d.nx < 2 || d.ny < 2 || d.nz < 2 || (d.nx - 1) % r || (d.ny - 1) % r || (d.nz - 1) % r)
      return bad("grid size not divisible by 2^(n_levels-1)");
    const long long nc = 2LL * ((d.nx - 1) / r + 1) * ((d.ny - 1) / r + 1) * ((d.nz - 1) / r + 1);
    if (nc > kMaxCoarse) return bad("coarsest grid too large for the dense coarse solve");
    if ((long long)d.nx * d.ny * d.nz * kPlanes > (1LL << 31)) return bad("grid too large");
    Group G;
    G.d = d;
    G.S = d.n_samples;
    G.s0 = s0;
    G.L = d.n_levels;
    s0 += G.S;
    pb->groups.push_back(G);
  }
  pb->S_total = s0;
  plan_pools(pb);
  for (Group& G : pb->groups) {
    edf_status s = alloc_group(pb, G);
    if (s) {
      std::fprintf(stderr, "edf_create_problem: %s\n", pb->err.c_str());
      edf_destroy(pb);
      return s;
    }
  }
  const bool shared_stream = opts->concurrent_groups == 2;
  for (Group& G : pb->groups) {
    const bool ok =
        (shared_stream && &G != &pb->groups[0]
             ? (G.st = pb->groups[0].st) != nullptr
             : hipStreamCreateWithFlags(&G.st, hipStreamNonBlocking) == hipSuccess) &&
        hipHostMalloc((void**)&G.h_int, sizeof(int) * G.S) == hipSuccess &&
        hipHostMalloc((void**)&G.h_list, sizeof(int) * G.S) == hipSuccess &&
        hipHostMalloc((void**)&G.h_dbl, sizeof(double) * G.S) == hipSuccess &&
        hipHostMalloc((void**)&G.h_ks, sizeof(KrylovScalars) * G.S) == hipSuccess;
    if (!ok || upload_initial(pb, G) != EDF_OK) {
      (void)hipGetLastError();
      edf_destroy(pb);
      return EDF_ERR_HIP;
    }
  }
  *out = pb;
  return EDF_OK;
}

edf_status edf_set_parameters(edf_problem* pb, const double* xi) {
  if (!pb) return EDF_ERR_ARG;
  const int nxi = pb->phys.n_xi;
  if (nxi > 0 && !xi) return fail(pb, EDF_ERR_ARG, "xi is NULL");
  for (size_t e = 0; e < (size_t)pb->S_total * nxi; ++e)
    if (!(std::fabs(xi[e]) <= 1.0)) return fail(pb, EDF_ERR_ARG, "|xi| > 1 or not finite");
  FieldParams fp{pb->phys.lx, pb->phys.ly, pb->phys.lz, pb->phys.phi_mean, pb->phys.K_mean,
                 pb->phys.field_model, nxi};
  const size_t ld = std::max(nxi, 1);
  const size_t cnt = (size_t)pb->S_total * ld;
  edf_status es;
  if (!pb->dxi && (es = dalloc(pb, &pb->dxi, cnt))) return es;
  if (!pb->dxi_new && (es = dalloc(pb, &pb->dxi_new, cnt))) return es;
  if (!pb->bad && (es = dalloc(pb, &pb->bad, (size_t)pb->S_total))) return es;
  std::vector<double> hx(cnt, 0.0);
  if (nxi > 0) std::memcpy(hx.data(), xi, (size_t)pb->S_total * nxi * sizeof(double));
  // the fields of every level are checked from the staged parameters before anything
  // of the problem changes
  EDF_TRY(hipStreamSynchronize(pb->st));
  EDF_TRY(hipMemcpyAsync(pb->dxi_new, hx.data(), cnt * sizeof(double), hipMemcpyHostToDevice, pb->st));
  launch_fill<int>(pb->bad, (size_t)pb->S_total, 1, nullptr, 0, pb->st);
  for (Group& G : pb->groups)
    for (Level& L : G.lv)
      launch_check_coefficients(L.g, fp, pb->dxi_new + (size_t)G.s0 * ld, G.S, pb->bad + G.s0, pb->st);
  EDF_CHECK_LAUNCH();
  std::vector<int> bad(pb->S_total);
  EDF_TRY(hipMemcpyAsync(bad.data(), pb->bad, bad.size() * sizeof(int), hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipStreamSynchronize(pb->st));
  for (int s = 0; s < pb->S_total; ++s)
    if (bad[s])
      return fail(pb, EDF_ERR_ARG, "sample " + std::to_string(s) +
                                       ": porosity outside (0,1) or permeability not positive");
  std::swap(pb->dxi, pb->dxi_new);
  for (Group& G : pb->groups)
    for (Level& L : G.lv)
      launch_coefficients(L.g, fp, pb->dxi + (size_t)G.s0 * ld, G.S, L.phi, L.K, pb->st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipStreamSynchronize(pb->st));
  for (Group& G : pb->groups) reset_history(G);
  pb->traj_valid = false;
  pb->params_set = true;
  return EDF_OK;
}

edf_status edf_set_state(edf_problem* pb, int32_t sample, const double* pc, int32_t is_dev) {
  if (!pb || !pc) return EDF_ERR_ARG;
  Group* G;
  int s;
  edf_status e;
  if ((e = find_sample(pb, sample, &G, &s))) return e;
  const hipMemcpyKind k = is_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  EDF_TRY(hipMemcpyAsync(G->u + s * G->n, pc, G->n * sizeof(double), k, pb->st));
  EDF_TRY(hipMemcpyAsync(G->u_old + s * G->n, pc, G->n * sizeof(double), k, pb->st));
  if (!is_dev) EDF_TRY(hipStreamSynchronize(pb->st));
  // a new state resets the sample: no failure, no sub-step history, counters from zero
  G->fail_status[s] = EDF_SAMPLE_OK;
  G->stats[s] = edf_step_stats{};
  if ((int)G->h_start.size() == G->S) {
    G->h_start[s] = 0;
    G->clean[s] = 0;
    G->wait[s] = kFirstWait;
    G->probing[s] = 0;
    G->pred_dt[s] = 0.0;
  }
  pb->traj_valid = false;
  return EDF_OK;
}

edf_status edf_get_state(edf_problem* pb, int32_t sample, double* pc, int32_t is_dev) {
  if (!pb || !pc) return EDF_ERR_ARG;
  Group* G;
  int s;
  edf_status e;
  if ((e = find_sample(pb, sample, &G, &s))) return e;
  const hipMemcpyKind k = is_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  EDF_TRY(hipMemcpyAsync(pc, G->u + s * G->n, G->n * sizeof(double), k, pb->st));
  if (!is_dev) EDF_TRY(hipStreamSynchronize(pb->st));
  return EDF_OK;
}

}  // extern "C"

namespace {

// one step of every group (edf_step without touching the recorded trajectory)
edf_status step_all(edf_problem* pb, double dt, edf_step_stats* stats) {
  EDF_TRY(hipStreamSynchronize(pb->st));  // work the caller queued before this step
  // the groups are independent and each steps on its own stream; with
  // concurrent_groups each also runs from its own host thread, so that one group's
  // host round trips and small launches overlap another's sweeps
  const size_t ng = pb->groups.size();
  std::vector<edf_status> rc(ng, EDF_OK);
  auto run = [&](size_t gi) {
    if (hipSetDevice(pb->device) != hipSuccess) {
      rc[gi] = fail(pb, EDF_ERR_HIP, "hipSetDevice failed in a group thread");
      return;
    }
    rc[gi] = macro_step(pb, pb->groups[gi], dt);
    if (hipStreamSynchronize(pb->groups[gi].st) != hipSuccess && rc[gi] == EDF_OK)
      rc[gi] = fail(pb, EDF_ERR_HIP, "group stream synchronisation failed");
  };
  if (ng == 1 || !pb->opts.concurrent_groups) {
    for (size_t gi = 0; gi < ng; ++gi) run(gi);
  } else {
    std::vector<std::thread> th;
    th.reserve(ng);
    for (size_t gi = 0; gi < ng; ++gi) th.emplace_back(run, gi);
    for (std::thread& t : th) t.join();
  }
  for (size_t gi = 0; gi < ng; ++gi)
    if (rc[gi] != EDF_OK) return rc[gi];
  bool all_failed = true;
  for (Group& G : pb->groups)
    for (int s = 0; s < G.S; ++s) {
      if (stats) stats[G.s0 + s] = G.stats[s];
      all_failed &= G.stats[s].status != EDF_SAMPLE_OK;
    }
  if (all_failed) return fail(pb, EDF_ERR_NO_CONVERGENCE, "every sample has failed");
  return EDF_OK;
}

}  // namespace

extern "C" {

edf_status edf_step(edf_problem* pb, double dt, edf_step_stats* stats) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (!(dt > 0) || !std::isfinite(dt)) return fail(pb, EDF_ERR_ARG, "dt must be positive");
  pb->traj_valid = false;
  return step_all(pb, dt, stats);
}

edf_status edf_solve(edf_problem* pb, double dt, int32_t n_steps, int32_t checkpoint_every,
                     edf_step_stats* stats) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (n_steps < 0) return fail(pb, EDF_ERR_ARG, "n_steps < 0");
  if (checkpoint_every < 0) return fail(pb, EDF_ERR_ARG, "checkpoint_every < 0");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(pb, EDF_ERR_ARG, "dt must be positive");
  pb->traj_valid = false;
  const int k = checkpoint_every;
  const bool record = k > 0 && n_steps > 0;
  if (record) {
    EDF_TRY(hipStreamSynchronize(pb->st));
    for (Group& G : pb->groups) {
      if ((e = ensure_trajectory_buffers(pb, G, n_steps, k))) return e;
      G.H.assign(n_steps, std::vector<int>(G.S, 0));
      G.traj_fail.assign(G.S, 0);
      for (int s = 0; s < G.S; ++s) G.traj_fail[s] = G.fail_status[s] != EDF_SAMPLE_OK;
      if ((e = scatter(pb, G, G.u, G.ckpt, G.ckpt_cap, std::vector<int>(G.S, 0)))) return e;
      EDF_TRY(hipStreamSynchronize(G.st));
    }
  }
  // the recorded steps start Newton from the state (the adjoint recomputes them so)
  struct Recording {
    edf_problem* pb;
    ~Recording() { pb->recording = false; }
  } rec_guard{pb};
  pb->recording = record;
  for (int m = 0; m < n_steps; ++m) {
    if ((e = step_all(pb, dt, m + 1 == n_steps ? stats : nullptr))) return e;
    if (!record) continue;
    for (Group& G : pb->groups) {
      for (int s = 0; s < G.S; ++s) {
        const edf_step_stats& t = G.stats[s];
        if (t.status != EDF_SAMPLE_OK) {
          G.traj_fail[s] = 1;
          continue;
        }
        int h = 0;
        while ((1 << h) < t.substeps) ++h;
        G.H[m][s] = h;
      }
      if ((m + 1) % k == 0 || m + 1 == n_steps) {
        const int slot = ceil_div(m + 1, k);
        if ((e = scatter(pb, G, G.u, G.ckpt, G.ckpt_cap, std::vector<int>(G.S, slot)))) return e;
        EDF_TRY(hipStreamSynchronize(G.st));
      }
    }
  }
  if (record) {
    pb->traj_valid = true;
    pb->traj_k = k;
    pb->traj_n = n_steps;
    pb->traj_dt = dt;
  }
  EDF_TRY(hipStreamSynchronize(pb->st));
  return EDF_OK;
}

edf_status edf_gpc_project(edf_problem* pb, int32_t group, int32_t cx, int32_t cy, int32_t cz,
                           int32_t degree, int32_t truncation, const double* weights,
                           int32_t* n_coef, double* coef, double* mean, double* var,
                           double* kernel_ms) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (group < 0 || group >= (int)pb->groups.size() || !weights || !n_coef || !mean || !var)
    return fail(pb, EDF_ERR_ARG, "bad gpc arguments");
  Group& G = pb->groups[group];
  const int M = pb->phys.n_xi, S = G.S;
  if (M < 1 || M > kGpcMaxM) return fail(pb, EDF_ERR_ARG, "the expansion needs 1..4 parameters");
  if (degree < 0 || degree > kGpcMaxDeg || (truncation != 0 && truncation != 1))
    return fail(pb, EDF_ERR_ARG, "degree must be in [0, 8] and truncation 0 or 1");
  const Geom& g = G.lv[0].g;
  if (cx < 2 || cy < 2 || cz < 2 || (g.nx - 1) % (cx - 1) || (g.ny - 1) % (cy - 1) ||
      (g.nz - 1) % (cz - 1))
    return fail(pb, EDF_ERR_ARG, "common grid not nested in the group's grid");
  for (int i = 0; i < S; ++i)
    if (!std::isfinite(weights[i])) return fail(pb, EDF_ERR_ARG, "weights not finite");
  // failed samples are left out, the others' weights renormalised to the same sum
  std::vector<double> wv(weights, weights + S);
  double w_all = 0.0, w_ok = 0.0;
  for (int i = 0; i < S; ++i) {
    w_all += wv[i];
    if (G.fail_status[i] != EDF_SAMPLE_OK) wv[i] = 0.0;
    w_ok += wv[i];
  }
  if (!(w_ok != 0.0)) return fail(pb, EDF_ERR_NO_CONVERGENCE, "no valid sample in the group");
  for (double& x : wv) x *= w_all / w_ok;
  std::vector<int> idx;
  gpc_indices(M, degree, truncation, idx);
  const int nc = (int)idx.size() / M;
  if (nc > kGpcMaxCoef) return fail(pb, EDF_ERR_ARG, "more than 128 expansion terms");
  std::vector<double> Q(nc);
  for (int q = 0; q < nc; ++q) {
    double a = 1.0;
    for (int j = 0; j < M; ++j) a /= 2.0 * idx[q * M + j] + 1.0;
    Q[q] = a;
  }
  const size_t Nc = (size_t)cx * cy * cz;
  hipStream_t st = pb->st;
  EDF_TRY(hipStreamSynchronize(st));
  if ((e = grow(pb, &pb->gpc_buf, &pb->gpc_cap, nc * Nc + nc + (size_t)nc * S + S + S * Nc + 2 * Nc)))
    return e;
  if ((e = grow(pb, &pb->gpc_ibuf, &pb->gpc_icap, (size_t)nc * M))) return e;
  double* C = pb->gpc_buf;
  double* dQ = C + nc * Nc;
  double* W = dQ + nc;
  double* dw = W + (size_t)nc * S;
  double* F = dw + S;
  double* mv = F + S * Nc;
  EDF_TRY(hipMemcpyAsync(pb->gpc_ibuf, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, st));
  EDF_TRY(hipMemcpyAsync(dQ, Q.data(), nc * sizeof(double), hipMemcpyHostToDevice, st));
  EDF_TRY(hipMemcpyAsync(dw, wv.data(), S * sizeof(double), hipMemcpyHostToDevice, st));
  launch_gather_common(g, cx, cy, cz, G.u, F, S, st);
  const int ldt = std::max(pb->phys.n_xi, 1);
  launch_gpc_weights(S, M, nc, pb->dxi + (size_t)G.s0 * ldt, ldt, dw, pb->gpc_ibuf, dQ, W, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms) {
    EDF_TRY(hipEventCreate(&e0));
    EDF_TRY(hipEventCreate(&e1));
  }
  launch_gpc_project(S, (int)Nc, nc, W, F, C, st, e0, e1);
  launch_gpc_moments((int)Nc, nc, C, dQ, mv, mv + Nc, st);
  EDF_CHECK_LAUNCH();
  if (coef) EDF_TRY(hipMemcpyAsync(coef, C, nc * Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipMemcpyAsync(mean, mv, Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipMemcpyAsync(var, mv + Nc, Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipStreamSynchronize(st));
  if (kernel_ms) {
    float ms = 0.f;
    EDF_TRY(hipEventElapsedTime(&ms, e0, e1));
    *kernel_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  *n_coef = nc;
  pb->gpc_nc = nc;
  pb->gpc_M = M;
  pb->gpc_deg = degree;
  pb->gpc_trunc = truncation;
  pb->gpc_Nc = (int)Nc;
  return EDF_OK;
}

edf_status edf_gpc_exceed(edf_problem* pb, int32_t n_points, const double* theta, double threshold,
                          double* prob, double* kernel_ms) {
  if (!pb || !theta || !prob || n_points < 1 || !std::isfinite(threshold))
    return fail(pb, EDF_ERR_ARG, "bad gpc exceedance arguments");
  if (pb->gpc_nc == 0) return fail(pb, EDF_ERR_STATE, "edf_gpc_project has not been called");
  const int M = pb->gpc_M, nc = pb->gpc_nc, Nc = pb->gpc_Nc;
  for (size_t e = 0; e < (size_t)n_points * M; ++e)
    if (!(std::fabs(theta[e]) <= 1.0)) return fail(pb, EDF_ERR_ARG, "points outside [-1,1]^M");
  // point chunks per block: at least 2048 points, at most 2^26 partial counts in all;
  // the basis table is built for batches of whole chunks, about 2^20 points at a time
  int chunk = 2048;
  while ((size_t)ceil_div(n_points, chunk) * Nc > (1u << 26)) chunk *= 2;
  const int n_chunks = ceil_div(n_points, chunk);
  const int batch_chunks = std::max(1, (1 << 20) / chunk);
  const int batch = std::min(n_chunks, batch_chunks) * chunk;  // a multiple of 64
  const int ncp = 4 * ((nc + 3) / 4);
  hipStream_t st = pb->st;
  edf_status e;
  EDF_TRY(hipStreamSynchronize(st));
  const size_t basis_off = ((size_t)n_points * M + Nc + 31) / 32 * 32;  // 256-byte aligned
  if ((e = grow(pb, &pb->gpc_pts, &pb->gpc_pcap, basis_off + (size_t)ncp * batch))) return e;
  if ((e = grow(pb, &pb->gpc_ibuf, &pb->gpc_icap, (size_t)nc * M + (size_t)n_chunks * Nc)))
    return e;
  double* pts = pb->gpc_pts;
  double* dprob = pts + (size_t)n_points * M;
  double* basis = pts + basis_off;
  int* idx = pb->gpc_ibuf;
  int* partial = idx + (size_t)nc * M;
  // the index table of the projection is written again: the buffer may have moved
  std::vector<int> table;
  gpc_indices(M, pb->gpc_deg, pb->gpc_trunc, table);
  EDF_TRY(hipMemcpyAsync(idx, table.data(), table.size() * sizeof(int), hipMemcpyHostToDevice, st));
  EDF_TRY(hipMemcpyAsync(pts, theta, (size_t)n_points * M * sizeof(double), hipMemcpyHostToDevice,
                         st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms) {
    EDF_TRY(hipEventCreate(&e0));
    EDF_TRY(hipEventCreate(&e1));
    EDF_TRY(hipEventRecord(e0, st));
  }
  // the surrogate's evaluation (basis tables and products) is timed as a whole
  for (int c0 = 0; c0 < n_chunks; c0 += batch_chunks) {
    const int nch = std::min(batch_chunks, n_chunks - c0);
    const int s0 = c0 * chunk;
    const int n = std::min(batch, n_points - s0);
    launch_gpc_basis(n, batch, nc, ncp, M, idx, pts + (size_t)s0 * M, basis, st);
    launch_gpc_exceed(Nc, nc, pb->gpc_buf, basis, batch, n, chunk, c0, nch, threshold, partial,
                      st, nullptr, nullptr);
  }
  if (kernel_ms) EDF_TRY(hipEventRecord(e1, st));
  launch_gpc_count(Nc, n_chunks, n_points, partial, dprob, st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(prob, dprob, Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipStreamSynchronize(st));
  if (kernel_ms) {
    float ms = 0.f;
    EDF_TRY(hipEventElapsedTime(&ms, e0, e1));
    *kernel_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return EDF_OK;
}

namespace {
// the statistics of edf_moments over the samples of every group (only < 0) or of group
// `only` alone; weights are indexed like those samples
edf_status moments_over(edf_problem* pb, int only, int32_t cx, int32_t cy, int32_t cz,
                        double threshold, const double* weights, double* mean, double* var,
                        double* exceed) {
  const size_t Nc = (size_t)cx * cy * cz;
  int S = 0;
  for (int gi = 0; gi < (int)pb->groups.size(); ++gi)
    if (only < 0 || gi == only) S += pb->groups[gi].S;
  std::vector<double> w(S);
  double sum = 0.0;
  int o = 0;
  for (int gi = 0; gi < (int)pb->groups.size(); ++gi) {
    if (only >= 0 && gi != only) continue;
    const Group& G = pb->groups[gi];
    for (int s = 0; s < G.S; ++s, ++o) {
      const double ws = weights ? weights[o] : 1.0 / S;
      w[o] = G.fail_status[s] == EDF_SAMPLE_OK ? ws : 0.0;
      sum += w[o];
    }
  }
  if (!(sum > 0)) return fail(pb, EDF_ERR_NO_CONVERGENCE, "no valid sample");
  for (double& x : w) x /= sum;
  const size_t need = Nc * (S + 3) + S;
  if (need > pb->mom_cap) {
    if (pb->mom_f) (void)hipFree(pb->mom_f);
    pb->mom_f = nullptr;
    EDF_TRY(hipMalloc(&pb->mom_f, need * sizeof(double)));
    pb->mom_cap = need;
  }
  double* f = pb->mom_f;
  double* dw = f + Nc * S;
  double* out = dw + S;
  EDF_TRY(hipMemcpyAsync(dw, w.data(), S * sizeof(double), hipMemcpyHostToDevice, pb->st));
  o = 0;
  for (int gi = 0; gi < (int)pb->groups.size(); ++gi) {
    if (only >= 0 && gi != only) continue;
    const Group& G = pb->groups[gi];
    launch_gather_common(G.lv[0].g, cx, cy, cz, G.u, f + (size_t)o * Nc, G.S, pb->st);
    o += G.S;
  }
  launch_moments((int)Nc, S, f, dw, threshold, out, out + Nc, out + 2 * Nc, pb->st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(mean, out, Nc * sizeof(double), hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipMemcpyAsync(var, out + Nc, Nc * sizeof(double), hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipMemcpyAsync(exceed, out + 2 * Nc, Nc * sizeof(double), hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipStreamSynchronize(pb->st));
  return EDF_OK;
}
}  // namespace

edf_status edf_moments(edf_problem* pb, int32_t cx, int32_t cy, int32_t cz, double threshold,
                       const double* weights, double* mean, double* var, double* exceed) {
  if (!pb || !mean || !var || !exceed) return EDF_ERR_ARG;
  if (cx < 2 || cy < 2 || cz < 2) return fail(pb, EDF_ERR_ARG, "common grid too small");
  for (Group& G : pb->groups) {
    const Geom& g = G.lv[0].g;
    if ((g.nx - 1) % (cx - 1) || (g.ny - 1) % (cy - 1) || (g.nz - 1) % (cz - 1))
      return fail(pb, EDF_ERR_ARG, "common grid not nested in every group");
  }
  return moments_over(pb, -1, cx, cy, cz, threshold, weights, mean, var, exceed);
}

edf_status edf_group_moments(edf_problem* pb, int32_t group, double threshold,
                             const double* weights, double* mean, double* var, double* exceed) {
  if (!pb || !mean || !var || !exceed) return EDF_ERR_ARG;
  if (group < 0 || group >= (int)pb->groups.size())
    return fail(pb, EDF_ERR_ARG, "group index out of range");
  const Geom& g = pb->groups[group].lv[0].g;
  return moments_over(pb, group, g.nx, g.ny, g.nz, threshold, weights, mean, var, exceed);
}

edf_status edf_moments_noalloc(edf_problem* pb, int32_t cx, int32_t cy, int32_t cz,
                               double threshold, const double* weights, double* mean, double* var,
                               double* exceed) {
  if (!pb || !mean || !var || !exceed) return EDF_ERR_ARG;
  if (cx < 2 || cy < 2 || cz < 2) return fail(pb, EDF_ERR_ARG, "common grid too small");
  for (Group& G : pb->groups) {
    const Geom& g = G.lv[0].g;
    if ((g.nx - 1) % (cx - 1) || (g.ny - 1) % (cy - 1) || (g.nz - 1) % (cz - 1))
      return fail(pb, EDF_ERR_ARG, "common grid not nested in every group");
  }
  const size_t Nc = (size_t)cx * cy * cz;
  const int S = pb->S_total;
  // scratch layout (doubles): weights [S], failure flags [S] (ints), their sum, the three
  // output fields [3 Nc], then the c fields of a chunk of samples [chunk][Nc]
  auto up32 = [](size_t a) { return (a + 31) / 32 * 32; };
  const size_t o_w = 0, o_flag = up32(S), o_sum = o_flag + up32((S + 1) / 2), o_out = o_sum + 32,
               o_f = o_out + up32(3 * Nc);
  if (o_f + Nc > kScratchDoubles)
    return fail(pb, EDF_ERR_ARG,
                "edf_moments_noalloc: " + std::to_string(S) + " samples and a common grid of " +
                    std::to_string(Nc) + " vertices need more than its scratch of " +
                    std::to_string(kScratchDoubles) + " doubles (use edf_moments)");
  double* base = (pb->device >= 0 && pb->device < kMaxDevices) ? g_scratch[pb->device] : nullptr;
  if (!base)
    return fail(pb, EDF_ERR_HIP, pb->device >= 0 && pb->device < kMaxDevices
                                     ? g_scratch_err[pb->device]
                                     : std::string("device index beyond the scratch table"));
  const int chunk = (int)std::min<size_t>((kScratchDoubles - o_f) / Nc, (size_t)S);
  hipStream_t st = pb->st;
  double* w = base + o_w;
  int* flag = reinterpret_cast<int*>(base + o_flag);
  double* out = base + o_out;
  double* f = base + o_f;
  // the weights (the caller's, or 1/S) and the failure flags, normalised on the device in
  // sample order as edf_moments does it on the host
  if (weights)
    EDF_TRY(hipMemcpyAsync(w, weights, S * sizeof(double), hipMemcpyHostToDevice, st));
  else
    launch_fill<double>(w, (size_t)S, 1, nullptr, 1.0 / S, st);
  for (Group& G : pb->groups)
    EDF_TRY(hipMemcpyAsync(flag + G.s0, G.fail_status.data(), G.S * sizeof(int),
                           hipMemcpyHostToDevice, st));
  launch_normalise_weights(S, w, flag, base + o_sum, st);
  double sum = 0.0;
  EDF_TRY(hipMemcpyAsync(&sum, base + o_sum, sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipStreamSynchronize(st));
  if (!(sum > 0)) return fail(pb, EDF_ERR_NO_CONVERGENCE, "no valid sample");
  for (int pass = 0; pass < 2; ++pass)
    for (int s0 = 0; s0 < S; s0 += chunk) {
      const int n = std::min(chunk, S - s0);
      for (Group& G : pb->groups) {  // the chunk's samples of every group, in sample order
        const int a = std::max(s0, G.s0), b = std::min(s0 + n, G.s0 + G.S);
        if (a < b)
          launch_gather_common(G.lv[0].g, cx, cy, cz, G.u + (size_t)(a - G.s0) * G.n,
                               f + (size_t)(a - s0) * Nc, b - a, st);
      }
      launch_moments_chunk(pass, (int)Nc, s0, n, f, w, threshold, out, out + Nc, out + 2 * Nc, st);
    }
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(mean, out, Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipMemcpyAsync(var, out + Nc, Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipMemcpyAsync(exceed, out + 2 * Nc, Nc * sizeof(double), hipMemcpyDeviceToHost, st));
  EDF_TRY(hipStreamSynchronize(st));
  return EDF_OK;
}

edf_status edf_residual(edf_problem* pb, int32_t sample, const double* u, const double* u_old,
                        double dt, double* F, int32_t is_dev) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (!u || !u_old || !F || !(dt > 0)) return fail(pb, EDF_ERR_ARG, "bad residual arguments");
  Group* G;
  int s;
  if ((e = find_sample(pb, sample, &G, &s))) return e;
  const size_t n = G->n;
  // the trial-state buffers of this sample serve as scratch
  double* du = G->ut + s * n;
  double* duo = G->kr + s * n;
  double* dF = G->Ft + s * n;
  const hipMemcpyKind kin = is_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  EDF_TRY(hipMemcpyAsync(du, u, n * sizeof(double), kin, pb->st));
  EDF_TRY(hipMemcpyAsync(duo, u_old, n * sizeof(double), kin, pb->st));
  const Level& L = G->lv[0];
  const Phys ph = make_phys(pb->phys, L.g, dt);
  launch_defect(L.g, ph, nullptr, L.phi + s * L.cells, L.K + s * L.cells, du, duo, dF, 1, nullptr,
                pb->st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(F, dF, n * sizeof(double),
                         is_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipStreamSynchronize(pb->st));
  return EDF_OK;
}

edf_status edf_get_jacobian(edf_problem* pb, int32_t sample, const double* u, double dt,
                            int32_t level, double* out) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (!u || !out || !(dt > 0)) return fail(pb, EDF_ERR_ARG, "bad jacobian arguments");
  Group* G;
  int s;
  if ((e = find_sample(pb, sample, &G, &s))) return e;
  if (level < 0 || level >= G->L) return fail(pb, EDF_ERR_ARG, "level out of range");
  const size_t n = G->n;
  double* du = G->ut + s * n;
  EDF_TRY(hipMemcpyAsync(du, u, n * sizeof(double), hipMemcpyHostToDevice, pb->st));
  // inject through scratch: coarse-level states of this sample
  const double* cur = du;
  for (int l = 1; l <= level; ++l) {
    double* dst = G->lv[l].u + s * 2 * (size_t)G->lv[l].g.N;
    launch_inject(G->lv[l - 1].g, G->lv[l].g, cur, dst, 1, nullptr, pb->st);
    cur = dst;
  }
  const Level& L = G->lv[level];
  const size_t N = L.g.N;
  double *A = nullptr, *nat = nullptr;
  EDF_TRY(hipMalloc(&A, kPlanes * (size_t)L.g.off[8] * sizeof(double)));
  EDF_TRY(hipMalloc(&nat, kPlanes * N * sizeof(double)));
  const Phys ph = make_phys(pb->phys, L.g, dt);
  launch_assemble(L.g, ph, nullptr, L.phi + s * L.cells, L.K + s * L.cells, cur, A, nullptr, 1,
                  nullptr, pb->st, false);
  launch_stencil_to_natural(L.g, A, nat, pb->st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(out, nat, kPlanes * N * sizeof(double), hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipStreamSynchronize(pb->st));
  EDF_TRY(hipFree(A));
  EDF_TRY(hipFree(nat));
  return EDF_OK;
}

edf_status edf_apply_vcycle(edf_problem* pb, int32_t group, double dt, const double* x,
                            double* y) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (group < 0 || group >= (int)pb->groups.size() || !x || !y || !(dt > 0))
    return fail(pb, EDF_ERR_ARG, "bad vcycle arguments");
  Group& G = pb->groups[group];
  EDF_TRY(hipStreamSynchronize(pb->st));
  set_dt(pb, G, dt);
  std::vector<int> all(G.S, 1);
  if ((e = upload_ints(pb, G, G.nmask, all))) return e;
  if ((e = set_sample_list(pb, G, all.data()))) return e;
  if ((e = assemble_all(pb, G, G.nmask, nullptr))) return e;
  EDF_TRY(hipMemcpyAsync(G.kp, x, G.S * G.n * sizeof(double), hipMemcpyHostToDevice, G.st));
  G.n_active = G.S;
  precondition(pb, G, G.kp, G.kph, G.nmask);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(y, G.kph, G.S * G.n * sizeof(double), hipMemcpyDeviceToHost, G.st));
  EDF_TRY(hipStreamSynchronize(G.st));
  return prof_flush(pb, G);
}

edf_status edf_apply_jacobian(edf_problem* pb, int32_t group, const double* x, double* y) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (group < 0 || group >= (int)pb->groups.size() || !x || !y)
    return fail(pb, EDF_ERR_ARG, "bad apply arguments");
  Group& G = pb->groups[group];
  EDF_TRY(hipMemcpyAsync(G.kp, x, G.S * G.n * sizeof(double), hipMemcpyHostToDevice, pb->st));
  JacOp J;
  if (pb->opts.matrix_free) {  // at the group's states with the last assembly's step
    J.ph = G.lv[0].ph;
    J.phi = G.lv[0].phi;
    J.K = G.lv[0].K;
    J.u = G.u;
  } else {
    J.A = G.lv[0].A64;
  }
  launch_spmv(G.lv[0].g, J, G.kp, G.kv, G.S, nullptr, pb->st);
  EDF_CHECK_LAUNCH();
  EDF_TRY(hipMemcpyAsync(y, G.kv, G.S * G.n * sizeof(double), hipMemcpyDeviceToHost, pb->st));
  EDF_TRY(hipStreamSynchronize(pb->st));
  return EDF_OK;
}

edf_status edf_adjoint(edf_problem* pb, const edf_qoi* qoi, double* J, double* dJ_dxi) {
  edf_status e;
  if ((e = check_ready(pb))) return e;
  if (!qoi || !J || !dJ_dxi) return fail(pb, EDF_ERR_ARG, "bad adjoint arguments");
  if (qoi->kind != 0) return fail(pb, EDF_ERR_ARG, "unknown quantity of interest");
  if (!(qoi->rtol >= 0.0 && qoi->rtol < 1.0)) return fail(pb, EDF_ERR_ARG, "rtol not in [0, 1)");
  if (pb->phys.field_model == EDF_FIELD_CONST || pb->phys.n_xi < 1)
    return fail(pb, EDF_ERR_ARG, "the constant field has no parameters");
  QoiBox b;
  for (int i = 0; i < 6; ++i) {
    if (!std::isfinite(qoi->box[i])) return fail(pb, EDF_ERR_ARG, "box not finite");
    b.b[i] = qoi->box[i];
  }
  if (!pb->traj_valid)
    return fail(pb, EDF_ERR_STATE, "no recorded trajectory: call edf_solve with checkpoint_every > 0 "
                                   "(and nothing that changes states or parameters) first");
  const int nxi = pb->phys.n_xi;
  EDF_TRY(hipStreamSynchronize(pb->st));
  for (Group& G : pb->groups) {
    std::vector<double> Jv, gr;
    const std::vector<edf_step_stats> keep = G.stats;  // the replays count Newton work
    e = adjoint_group(pb, G, b, qoi->rtol > 0.0 ? qoi->rtol : kAdjointRtol, Jv, gr);
    G.stats = keep;
    if (e) return e;
    for (int s = 0; s < G.S; ++s) {
      J[G.s0 + s] = Jv[s];
      for (int m = 0; m < nxi; ++m)
        dJ_dxi[(size_t)(G.s0 + s) * nxi + m] = m < 4 ? gr[4 * s + m] : 0.0;
    }
  }
  return EDF_OK;
}

edf_status edf_autotune(edf_problem* pb, double dt) {
  edf_status e = check_ready(pb);
  if (e) return e;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(pb, EDF_ERR_ARG, "dt must be positive");
  EDF_TRY(hipStreamSynchronize(pb->st));
  const bool joint = pb->opts.concurrent_groups == 2 && pb->groups.size() > 1;
  for (Group& G : pb->groups) {
    set_dt(pb, G, dt);
    if ((e = autotune_group(pb, G, true, !joint))) return fail(pb, e, "autotuning failed");
  }
  if (joint) {
    // merged V-cycles share a bottom launch only between groups that fuse the same
    // grids: one number d of fused levels for all groups (their coarsest grids are the
    // same whenever their hierarchies line up), the d with the least summed time
    int dmax = 1 << 30;
    for (Group& G : pb->groups) dmax = std::min(dmax, G.L - first_fusable(G));
    int best_d = 1;
    double best = -1.0;
    for (int d = 1; d <= dmax; ++d) {
      double t = 0.0;
      for (Group& G : pb->groups) t += G.tune_ms[G.L - d];
      if (best < 0 || t < best) {
        best = t;
        best_d = d;
      }
    }
    for (Group& G : pb->groups) {
      G.fuse_from = G.L - best_d;
      if ((e = autotune_group(pb, G, false, true))) return fail(pb, e, "autotuning failed");
    }
  }
  return EDF_OK;
}

edf_status edf_get_tuning(edf_problem* pb, int32_t group, int32_t* fuse_from, double* ms) {
  if (!pb || group < 0 || group >= (int)pb->groups.size() || !fuse_from)
    return fail(pb, EDF_ERR_ARG, "bad tuning arguments");
  Group& G = pb->groups[group];
  *fuse_from = G.fuse_from >= 0 ? G.fuse_from : default_fuse_from(G);
  if (ms)
    for (int l = 0; l < G.L; ++l) ms[l] = l < (int)G.tune_ms.size() ? G.tune_ms[l] : -1.0;
  return EDF_OK;
}

edf_status edf_set_tuning(edf_problem* pb, int32_t group, int32_t fuse_from) {
  if (!pb || group < 0 || group >= (int)pb->groups.size())
    return fail(pb, EDF_ERR_ARG, "bad tuning arguments");
  Group& G = pb->groups[group];
  if (fuse_from < first_fusable(G) || fuse_from >= G.L)
    return fail(pb, EDF_ERR_ARG, "fuse_from must lie between the first level of at most 4096 "
                                 "vertices (at most 6 fused levels) and the coarsest level");
  G.fuse_from = fuse_from;
  return EDF_OK;
}

edf_status edf_get_line_tiles(edf_problem* pb, int32_t group, int32_t* cols) {
  if (!pb || !cols || group < 0 || group >= (int)pb->groups.size())
    return fail(pb, EDF_ERR_ARG, "bad tile arguments");
  const Group& G = pb->groups[group];
  for (int l = 0; l < G.L; ++l) cols[l] = G.lv[l].LF ? G.lv[l].line_cols : 0;
  return EDF_OK;
}

edf_status edf_set_line_tiles(edf_problem* pb, int32_t group, const int32_t* cols) {
  if (!pb || !cols || group < 0 || group >= (int)pb->groups.size())
    return fail(pb, EDF_ERR_ARG, "bad tile arguments");
  Group& G = pb->groups[group];
  const bool mx = mixed(pb);
  for (int l = 0; l < G.L; ++l) {
    if (!G.lv[l].LF) {
      if (cols[l] != 0) return fail(pb, EDF_ERR_ARG, "a level without line smoothing takes 0");
      continue;
    }
    if (!(mx ? line_cols_valid<float>(G.lv[l].g, cols[l])
             : line_cols_valid<double>(G.lv[l].g, cols[l])))
      return fail(pb, EDF_ERR_ARG, "columns per workgroup must be 8, 16 or 32 and fit the LDS");
  }
  for (int l = 0; l < G.L; ++l)
    if (G.lv[l].LF) G.lv[l].line_cols = cols[l];
  return EDF_OK;
}

edf_status edf_profile(edf_problem* pb, int32_t enable, double* out) {
  if (!pb) return EDF_ERR_ARG;
  edf_status e;
  if (out)
    for (int q = 0; q < 16; ++q) out[q] = 0.0;
  for (Group& G : pb->groups) {
    if ((e = prof_flush(pb, G))) return e;
    if (out) {
      for (int k = 0; k < 2; ++k) {
        out[3 * k + 0] += G.prof_count[k];
        out[3 * k + 1] += G.prof_ms[k];
        out[3 * k + 2] += G.prof_bytes[k];
      }
      out[6] += G.prof_all_count[0];
      out[7] += G.prof_all_bytes[0];
      out[8] += G.prof_count[2];
      out[9] += G.prof_ms[2];
      out[10] += G.prof_bytes[2];
      out[11] += G.prof_all_count[1];
      out[12] += G.prof_all_bytes[1];
      out[13] += G.prof_count[3];
      out[14] += G.prof_ms[3];
      out[15] += G.prof_bytes[3];
    }
    if (enable) {
      for (int k = 0; k < 4; ++k) G.prof_count[k] = G.prof_ms[k] = G.prof_bytes[k] = 0;
      for (int k = 0; k < 2; ++k) G.prof_all_count[k] = G.prof_all_bytes[k] = 0;
      G.prof_tick = 0;
    }
    G.prof_on = enable != 0;
  }
  return EDF_OK;
}

const char* edf_last_error(const edf_problem* pb) { return pb ? pb->err.c_str() : "null problem"; }

void edf_destroy(edf_problem* pb) {
  if (!pb) return;
  if (pb->st) (void)hipStreamSynchronize(pb->st);
  std::vector<hipStream_t> destroyed;  // groups may share one stream (concurrent_groups = 2)
  for (Group& G : pb->groups) {
    if (G.st && std::find(destroyed.begin(), destroyed.end(), G.st) == destroyed.end()) {
      (void)hipStreamSynchronize(G.st);
      (void)hipStreamDestroy(G.st);
      destroyed.push_back(G.st);
    }
    for (hipEvent_t e : G.prof_ev) (void)hipEventDestroy(e);
    for (auto& v : G.vgraphs) (void)hipGraphExecDestroy(v.exec);
    if (G.h_int) (void)hipHostFree(G.h_int);
    if (G.h_list) (void)hipHostFree(G.h_list);
    if (G.h_dbl) (void)hipHostFree(G.h_dbl);
    if (G.h_ks) (void)hipHostFree(G.h_ks);
    if (G.ckpt) (void)hipFree(G.ckpt);
    if (G.seg) (void)hipFree(G.seg);
  }
  for (void* p : pb->allocs) (void)hipFree(p);
  if (pb->mom_f) (void)hipFree(pb->mom_f);
  if (pb->gpc_buf) (void)hipFree(pb->gpc_buf);
  if (pb->gpc_ibuf) (void)hipFree(pb->gpc_ibuf);
  if (pb->gpc_pts) (void)hipFree(pb->gpc_pts);
  delete pb;
}

}  // extern "C"
