// Library context and host-side helpers shared by the forward (api.hip) and
// reverse (adjoint.hip) orchestration.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "sdc.h"

namespace sdc {

static_assert(kRecDiag >= kMaxDiag, "block records must hold every diagonal offset");

struct MapBuf {
  BlkRec* rec = nullptr;
  int32_t* inst_blk0 = nullptr;
  int32_t* inst_nblk = nullptr;
  int32_t* inst_cnt = nullptr;
  int64_t* inst_nnz = nullptr;
  int32_t* aoff = nullptr;
  int32_t* totals = nullptr;
  const int32_t* idx = nullptr;       // padded list the map indexes (null: all rows)
  // host mirror, valid after the map is built
  int32_t nblk = 0;
  int32_t n_inst = 0;
  int32_t cap = 0;                    // entries the record array holds
  int32_t xcd_shift = kXcdContig;     // order of the entries over the XCDs (see Map)
  int32_t max_nb = 0;                 // most blocks of one instance
  int64_t rows = 0;
  std::vector<int32_t> cnt;
  std::vector<int64_t> nnz;

  Map dev() const { return Map{rec, inst_blk0, inst_nblk, idx, nblk, n_inst, nullptr, xcd_shift}; }
  // the per-instance totals pass: for instances over kTotBlocks blocks, and
  // on maps long enough (over kTotMapBlocks blocks, i.e. launches that
  // stream from HBM) that one more launch costs less than every block
  // re-reading its instance's partials (instances over kTotMinBlocks)
  double* tot_if_large(double* tot) const {
    return max_nb > kTotBlocks || (nblk > kTotMapBlocks && max_nb > kTotMinBlocks) ? tot : nullptr;
  }
  // listed sets whose instances have at most kTotBlocks blocks: the CG
  // launches sum their partials themselves after the stencil sums instead of
  // a totals pass before them
  bool late_partials() const { return idx && max_nb <= kTotBlocks; }
  NextMap next(const int64_t* node_off, const int32_t* dia_off, int nd) const {
    return NextMap{rec, inst_blk0, inst_nblk, inst_cnt, inst_nnz, aoff, totals, node_off, dia_off, nd, cap};
  }
};

struct Stimulus {
  double t_on;
  int32_t* nodes;
  int64_t n;
  double value;
};

// Whether stimulus s belongs to the step [t, t + dt): it overwrites the state
// at the start of the step that contains its time.  Both ends of the
// interval are moved down by 1e-9 dt, so that a time on a step boundary goes
// to the step starting there even when the caller's t was accumulated with
// rounding just above it.  The one rule for the forward step, the
// first-sweep set and the reverse step.
inline bool stimulus_applies(const Stimulus& s, double t, double dt) {
  return t - 1e-9 * dt <= s.t_on && s.t_on < t + dt - 1e-9 * dt;
}

}  // namespace sdc

using sdc::Collocation;
using sdc::CollArgs;
using sdc::HostSystem;
using sdc::MapBuf;
using sdc::Stimulus;
using sdc::CgState;
using sdc::Mat;
using sdc::NextMap;
using sdc::EmiArgs;
using sdc::BlkRec;
using sdc::ZeroVecs;
using sdc::kScal;
using sdc::CgStop;
using sdc::kMaxDelay;

struct sdc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<void*> allocs;

  bool ready = false;
  sdc_params prm{};
  Collocation col{};
  CollArgs cargs{};
  int dim = 0;
  int64_t N = 0, nnz = 0;
  int n_inst = 0;
  std::vector<int64_t> node_off_h;
  HostSystem host;   // kept for sdc_get_system

  int32_t *rowptr = nullptr, *colidx = nullptr, *diagpos = nullptr;
  double *Aval = nullptr, *Hval = nullptr, *ml = nullptr, *dinv = nullptr;
  // diagonal storage (nd > 0 when every instance has at most kMaxDiag offsets)
  int nd = 0;
  int32_t xcd_shift = sdc::kXcdContig;   // order of map entries over the XCDs, from the matrix bandwidth
  int32_t* dia_off = nullptr;      // [n_inst][nd]
  std::vector<int32_t> dia_off_h;
  double *dia_A = nullptr, *dia_H = nullptr;   // [nd/2+1][N], [M][nd/2+1][N] (offsets >= 0)
  bool use_dia = false;
  double t_csr_us = 0.0, t_dia_us = 0.0;
  // sliced ELL copy of A and every H_m (not with the linearized scheme, whose
  // sweeps rewrite the diagonals of the CSR and diagonal copies)
  int32_t* sell_ptr = nullptr;   // [nslice + 1] slice offsets (entries)
  int32_t* sell_col = nullptr;   // [sell_len] columns, padding = the row
  double* sell_A = nullptr;      // [sell_len]
  double* sell_H = nullptr;      // [M][sell_len]
  int64_t sell_len = 0;
  int nslice = 0;
  bool use_sell = false;
  double t_sell_us = 0.0;
  // all-rows CG launches with diagonal storage: two rows per thread (else
  // one), and the setup timings of one and two rows per thread (0: not timed)
  bool pair_all = true;
  double t_rows_us[2] = {0.0, 0.0};
  int64_t* node_off_d = nullptr;
  double* ionic_d = nullptr;
  // cell-by-cell model (see sdc_emi): membrane partner, signed site length,
  // CSR position of the partner column and the off-diagonal membrane mass
  bool emi = false;
  double emi_cm = 0.0;
  int32_t* emi_part = nullptr;
  double* emi_sl = nullptr;
  int32_t* emi_ppos = nullptr;
  double* emi_pmass = nullptr;

  double *v0 = nullptr, *w0 = nullptr, *v = nullptr, *w = nullptr, *I = nullptr, *R = nullptr;
  double *Phi = nullptr, *Gam = nullptr, *dv = nullptr, *dI = nullptr, *dR = nullptr;
  double* amax = nullptr;
  // CG vectors: p and the iterate (dv[m]) are read on own rows only; r, w, s
  // are double-buffered because the SpMV reads them at neighbouring columns
  double* p = nullptr;
  double* wg_p = nullptr;   // search direction of the one-workgroup solves (zero between solves)
  int64_t max_row = 0;      // most stored entries in a row of A
  // rows per thread of the one-workgroup solves: a property of the pattern,
  // so that both storages of a matrix solve alike
  int wg_rows_per_thread() const { return max_row <= 8 ? 2 : 1; }
  double *r[2] = {nullptr, nullptr}, *wv[2] = {nullptr, nullptr}, *s[2] = {nullptr, nullptr};

  double* cg_scal[2] = {nullptr, nullptr};   // [n_inst][kScal] by launch parity
  double* cg_tot = nullptr;                  // [n_inst][4] partial-sum totals (large instances)
  double* part[2] = {nullptr, nullptr};      // [nblk][4] by launch parity
  int32_t *cg_done = nullptr, *cg_iters = nullptr, *cg_blk_done = nullptr;
  int32_t *sel_cnt = nullptr, *sel_nnz = nullptr;

  MapBuf all;
  MapBuf dyn[2];
  int32_t* list[2] = {nullptr, nullptr};   // padded lists of dyn[0], dyn[1]: [nblk of all][kBlock]
  int cur = -1;   // -1: all rows; 0/1: dyn slot

  int32_t* h_i32 = nullptr;   // pinned staging
  int64_t* h_i64 = nullptr;

  std::vector<Stimulus> stims;
  std::vector<int32_t*> pin;
  std::vector<int64_t> pin_n;

  // host copy of the mesh (element data of the reverse step)
  std::vector<double> coords_h, tensor_h;
  std::vector<int32_t> elems_h;
  int64_t n_elem = 0;

  // reverse-step storage, allocated on first use
  struct Recording {                 // one recomputed step
    double *v = nullptr, *w = nullptr, *dv = nullptr;   // [K+1][M][N], [K+1][M][N], [K][M][N]
    int32_t* list = nullptr;                            // [K][N] active lists
    std::vector<int64_t> n;                             // rows per sweep, -1: all rows
    double t = 0.0;
    bool valid = false;
  };
  struct Adjoint {
    bool ready = false;
    int32_t *elems = nullptr, *nptr = nullptr, *nel = nullptr;
    double* pairw = nullptr;
    std::vector<Recording> slots;
    double *Lv = nullptr, *Lw = nullptr, *Ldv = nullptr, *Ldw = nullptr;
    double *Lv0 = nullptr, *Lw0 = nullptr, *psi = nullptr, *u = nullptr, *ga_row = nullptr, *qe = nullptr;
    uint8_t* in_set = nullptr;
  } adj;

  bool in_step = false;
  int k = 0;
  // CG updates of the last sweep's restricted solves, [M][n_inst] (empty before any sweep)
  std::vector<int32_t> last_iters;
  double* record_dv = nullptr;   // when set, a sweep copies its corrections here before the selection
  // per-node CG outcome of the current sweep, snapshot on the device (async steps)
  int32_t* hist_done = nullptr;    // [M][n_inst]
  int32_t* hist_iters = nullptr;   // [M][n_inst]
  int64_t redone_steps = 0;
  // Time of the step that would continue the last one begun (t + dt), and
  // whether the current step's t differs from it (the first step, a restart
  // from a checkpoint, a window run again): the CG budgets predicted from
  // the last step's iteration counts then belong to another time, and the
  // step takes the synchronous CG loop instead of risking a redo.
  double t_next = 0.0;
  bool t_known = false;
  bool t_jump = true;
  // energy-norm termination (prm.tol_sdc > 0)
  double* e_part = nullptr;        // [M][nblk of all] per-block energies of the sweep
  double* inst_energy = nullptr;   // [n_inst]
  int32_t* inst_stop = nullptr;    // [n_inst] instance stopped in this step
  double* h_term = nullptr;        // pinned: energies [n_inst], then stop flags (int32)
  bool all_stopped = false;
  bool terminate() const { return prm.tol_sdc > 0.0; }
  // a-priori drop tolerance (drop_mode 1): per instance, from each step's first sweep
  double* drop_part = nullptr;     // [nblk of all][2] per-block max |dv| and min dI/dv
  double* drop_theta = nullptr;    // [n_inst] TOL_drop of the current step
  double* drop_info = nullptr;     // [n_inst][4] TOL_drop, r, c, eta
  bool apriori_drop() const { return prm.drop_mode == 1; }
  // linearized scheme (scheme 1): lumped reaction Jacobian of the sweep
  double* G = nullptr;             // [M][N] ML dI/dv(v_m, w_m) at the sweep's iterate
  bool linearized() const { return prm.scheme == 1; }
  int k_min() const { return std::max(1, std::min(prm.K_min, prm.K)); }

  // heuristic first-sweep set (prm.first_rings > 0)
  int32_t* carry_list = nullptr;     // [N] the set the last step carried (ascending)
  int64_t carry_n = -1;              // its length; -1: none (next first sweep on all rows)
  int32_t* first_list = nullptr;     // [N] the current step's first-sweep set
  int64_t first_n = -1;              // its length; -1: all rows
  int64_t step_count = 0;            // steps begun since setup or the last reset
  double* mark[2] = {nullptr, nullptr};   // [N] row marks, ping-pong over the rings
  bool first_subset() const { return prm.first_rings > 0; }
  CgStop cg_stop() const {
    const bool e = prm.cg_energy_tol > 0.0;
    return CgStop{prm.cg_rtol * prm.cg_rtol, e ? prm.cg_energy_tol * prm.cg_energy_tol : 0.0, prm.cg_maxit,
                  e ? prm.cg_delay : 0};
  }

  // graph-captured sweeps (sdc_set_graph): sweep k of a step is one graph
  // with a fixed launch sequence: its CG solves take gbudget[k][m] launches
  // (launches after convergence return at once), the maps of sweeps k >= 1
  // are read through their live entry counts with grids of the all-rows
  // capacity, and the outcome goes to device history that the host reads
  // once per step
  bool graph_mode = false;
  bool graph_ready = false;
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraphExec_t> gexec;   // [K]
  std::vector<int> gbudget;            // [K][M]
  std::vector<int> gcap;               // [K] grid of sweep k (k >= 1): map entries the graph covers
  std::vector<int> seen_nblk;          // [K] map entries of sweep k in the last step (eager or graph)
  std::vector<int> seen_prev;          // [K] the same one step earlier
  void note_seen(int k, int nblk) {
    if (static_cast<int>(seen_nblk.size()) <= k) seen_nblk.resize(k + 1, all.nblk);
    if (static_cast<int>(seen_prev.size()) <= k) seen_prev.resize(k + 1, all.nblk);
    seen_prev[k] = seen_nblk[k];
    seen_nblk[k] = nblk;
  }
  int32_t* ghist = nullptr;            // device [K][M][n_inst] done, then [K][M][n_inst] iters
  int32_t* gh_hist = nullptr;          // pinned copy of ghist
  int64_t* gh_sizes = nullptr;         // pinned [K][map_sizes_words]: the sizes of each sweep's map
  std::vector<hipEvent_t> gev;         // K + 1 events around the sweeps of a graph step
  int64_t graph_steps = 0, graph_captures = 0, graph_redone = 0;
  bool graph_usable() const {
    bool pinned = false;
    for (auto* q : pin) pinned = pinned || q;
    return graph_mode && !pinned && !prof;
  }

  // kernel timing (bench only)
  bool prof = false;
  std::vector<hipEvent_t> ev;   // 2 per CG iteration launch
  hipEvent_t sweep_ev[2] = {nullptr, nullptr};   // around a sweep whose statistics are asked for
  sdc_profile_stats pst{};
  std::vector<int> pred;   // predicted CG iterations [3][SDC_MAX_SWEEPS][M]
  // Margin of an asynchronous CG budget over its prediction.  A solve whose
  // count rose by two or more from the last step's (for the same sweep and
  // node) overruns a budget of the prediction plus one, and its step is
  // redone.  Such rises are recorded per step (steps that continue the last
  // one only): while at least two of the last 64 steps had one, budgets get
  // max(2, pred / 16) launches of margin, else one.  The record does not
  // depend on the margin, and launches after convergence return at once,
  // so the margin changes no result, only how often a step is redone.
  uint64_t rise_steps = 0;   // bit j: the step j + 1 steps back had a rise
  bool rise_now = false;     // the current step has one
  bool wide_margin() const { return __builtin_popcountll(rise_steps) >= 2; }
  int budget_margin(int p) const { return wide_margin() ? std::max(2, p / 16) : 1; }
  // a solve's new count (mx updates) against the slot's prediction
  void note_count(int slot, int mx) {
    if (!t_jump && mx > pred[slot]) rise_now = true;
  }
  // prediction slot of node m in the current sweep: steps whose first sweep
  // takes all rows while heuristic first-sweep sets are on keep their own
  // history (their solves differ from the other steps')
  int pred_slot(int m) const {
    const int fam = first_subset() && first_n < 0 ? 2 : 0;
    return (fam * SDC_MAX_SWEEPS + std::min(k, SDC_MAX_SWEEPS - 1)) * prm.M + m;
  }

  const MapBuf& curmap() const { return cur < 0 ? all : dyn[cur]; }
  // output description for building a map into mb (records carry the diagonal offsets)
  NextMap next(const MapBuf& mb) const { return mb.next(node_off_d, nd > 0 ? dia_off : nullptr, nd); }
  CgState cg() const { return CgState{cg_done, cg_iters, cg_blk_done}; }
  // storage: 1 CSR, 2 diagonal, 3 sliced ELL
  Mat matA(int fmt) const {
    Mat a{rowptr, colidx, Aval, dia_off, dia_A, node_off_d, fmt == 2 ? nd : 0};
    if (fmt == 3) a.sptr = sell_ptr, a.scol = sell_col, a.sval = sell_A;
    return a;
  }
  Mat matH(int m, int fmt) const {
    Mat h{rowptr, colidx, Hval + static_cast<int64_t>(m) * nnz, dia_off,
          dia_H ? dia_H + static_cast<int64_t>(m) * (nd / 2 + 1) * N : nullptr, node_off_d, fmt == 2 ? nd : 0};
    if (fmt == 3) h.sptr = sell_ptr, h.scol = sell_col, h.sval = sell_H + static_cast<int64_t>(m) * sell_len;
    return h;
  }
  int fmt() const { return use_dia ? 2 : use_sell ? 3 : 1; }
  Mat A() const { return matA(fmt()); }
  Mat H(int m) const { return matH(m, fmt()); }
  ZeroVecs zv() const {
    return ZeroVecs{{r[0], r[1], wv[0], wv[1], s[0], s[1]}, dv, prm.M, N, emi ? dI : nullptr, emi ? dR : nullptr};
  }
  EmiArgs emi_args() const { return EmiArgs{emi ? emi_part : nullptr, emi_sl, emi_cm}; }
};


namespace sdc {

int fail(sdc_ctx* c, int code, const char* fmt, ...);

#define HIPC(call)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::sdc::fail(ctx, SDC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define TRY(x)                     \
  do {                             \
    int rc_ = (x);                 \
    if (rc_ != SDC_OK) return rc_; \
  } while (0)

template <class T>
int dalloc(sdc_ctx* ctx, T** out, size_t count) {
  void* ptr = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) return fail(ctx, SDC_ERR_OOM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  e = hipMemsetAsync(ptr, 0, bytes, ctx->stream);
  if (e != hipSuccess) return fail(ctx, SDC_ERR_HIP, "hipMemsetAsync: %s", hipGetErrorString(e));
  ctx->allocs.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return SDC_OK;
}

int alloc_map(sdc_ctx* ctx, MapBuf* mb, int32_t nblk_cap);
int fetch_map(sdc_ctx* ctx, MapBuf* mb);
int map_list(sdc_ctx* ctx, int slot, const int32_t* idx, int64_t n);
int run_cg(sdc_ctx* ctx, int m, const MapBuf& mb, double* x, int pred_slot, std::vector<int>* iters);
int do_sweep(sdc_ctx* ctx, sdc_sweep_stats* st, bool select_next, bool async = false,
             bool* short_budget = nullptr);
int restart_step(sdc_ctx* ctx);
int check_ready(sdc_ctx* ctx);
int emi_host_setup(sdc_ctx* ctx, const sdc_emi* emi, std::vector<int32_t>* part, std::vector<double>* sl,
                   std::vector<int32_t>* ppos, std::vector<double>* pmass);

}  // namespace sdc
