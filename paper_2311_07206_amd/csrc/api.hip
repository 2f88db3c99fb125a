// C ABI and host orchestration of the adaptive SDC step (see include/sdc.h).
//
// One context owns: the assembled system (CSR of A, lumped mass ML, the M
// node matrices H_m = ML + dt*QI[m][m]*A with their inverse diagonals), the
// collocation state [M][N] (v, w, I, R, Phi, Gam, dv, dI, dR), the CG work
// vectors, and the work maps of the active sets.  All device work goes to
// the context's stream; the host synchronises once per CG budget (to learn
// which instances converged) and once per selection (to size the next
// sweep's grids).
#include "sdc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "context.hpp"
#include "internal.hpp"
#include "kernels.hpp"

using namespace sdc;

namespace sdc {

int fail(sdc_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  c->err = buf;
  return code;
}

// The sizes a built map reports to the host, in one block so that one copy
// reads them: int64 inst_nnz[ni + 1], int32 totals[4], int32 inst_cnt[ni + 1].
size_t map_sizes_words(int ni) { return static_cast<size_t>(ni + 1) + 2 + (ni + 2) / 2; }

int alloc_map(sdc_ctx* ctx, MapBuf* mb, int32_t nblk_cap) {
  const int ni = ctx->n_inst;
  TRY(dalloc(ctx, &mb->rec, nblk_cap));
  TRY(dalloc(ctx, &mb->inst_blk0, ni + 1));
  TRY(dalloc(ctx, &mb->inst_nblk, ni + 1));
  int64_t* sizes = nullptr;
  TRY(dalloc(ctx, &sizes, map_sizes_words(ni)));
  mb->inst_nnz = sizes;
  mb->totals = reinterpret_cast<int32_t*>(sizes + ni + 1);
  mb->inst_cnt = mb->totals + 4;
  TRY(dalloc(ctx, &mb->aoff, ni + 1));
  mb->cnt.assign(ni, 0);
  mb->nnz.assign(ni, 0);
  mb->n_inst = ni;
  mb->cap = nblk_cap;
  mb->xcd_shift = ctx->xcd_shift;
  return SDC_OK;
}

// The host mirror of a map from its sizes block (map_sizes_words int64 words
// as the map's builder wrote them).
int parse_map_sizes(sdc_ctx* ctx, MapBuf* mb, const int64_t* words) {
  const int ni = ctx->n_inst;
  const int32_t* tot = reinterpret_cast<const int32_t*>(words + ni + 1);
  mb->nblk = tot[0];
  mb->rows = tot[1];
  if (tot[2] != 0)
    return fail(ctx, SDC_ERR_ARG, tot[2] == 1 ? "index list not strictly ascending or out of range"
                                             : "work map larger than its capacity");
  mb->max_nb = 0;
  for (int i = 0; i < ni; ++i) {
    mb->cnt[i] = tot[4 + i];
    mb->nnz[i] = words[i];
    mb->max_nb = std::max(mb->max_nb, (mb->cnt[i] + kBlock - 1) / kBlock);
  }
  return SDC_OK;
}

// Read a freshly built map's sizes back to the host (synchronises).
int fetch_map(sdc_ctx* ctx, MapBuf* mb) {
  const int ni = ctx->n_inst;
  HIPC(hipMemcpyAsync(ctx->h_i64, mb->inst_nnz, map_sizes_words(ni) * sizeof(int64_t), hipMemcpyDeviceToHost,
                      ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  return parse_map_sizes(ctx, mb, ctx->h_i64);
}

// Add the event timings of iterations [it0, it0 + budget) to the profile;
// an iteration counts for the instances whose CG had not stopped before it.
// Add the event timings of launches ev[2*(base+b)], ev[2*(base+b)+1] for
// iterations b = 0..budget-1 of one solve (iteration it0 + b); an iteration
// counts for the instances whose CG had not stopped before it.
int account_timing_at(sdc_ctx* ctx, const MapBuf& mb, int base, int budget, const int32_t* iters,
                      int it0 = 0) {
  const bool ident = mb.idx == nullptr;
  for (int b = 0; b < budget; ++b) {
    const int it = it0 + b;
    double bytes = 0.0, rows = 0.0, nnz = 0.0;
    for (int i = 0; i < ctx->n_inst; ++i) {
      if (it >= iters[i] || mb.cnt[i] == 0) continue;
      bytes += 8.0 * static_cast<double>(mb.nnz[i]) + (ident ? 88.0 : 92.0) * mb.cnt[i];
      rows += mb.cnt[i];
      nnz += static_cast<double>(mb.nnz[i]);
    }
    if (bytes == 0.0) continue;
    float t = 0.f;
    HIPC(hipEventElapsedTime(&t, ctx->ev[2 * (base + b)], ctx->ev[2 * (base + b) + 1]));
    ctx->pst.cg_launches++;
    ctx->pst.cg_ms += t;
    ctx->pst.cg_bytes += bytes;
    ctx->pst.cg_rows += rows;
    ctx->pst.cg_nnz += nnz;
    if (ident) {
      ctx->pst.cg_all_launches++;
      ctx->pst.cg_all_ms += t;
      ctx->pst.cg_all_bytes += bytes;
      ctx->pst.cg_all_rows += rows;
      ctx->pst.cg_all_nnz += nnz;
    }
  }
  return SDC_OK;
}

int account_timing(sdc_ctx* ctx, const MapBuf& mb, int it0, int budget, const int32_t* iters) {
  return account_timing_at(ctx, mb, 0, budget, iters, it0);
}

// Maps whose instances each hold at most small_set_rows rows (default and
// cap: what one workgroup takes, kWgThreads times its rows per thread) are
// solved by one workgroup per instance in a single launch.
bool wg_solve(const sdc_ctx* ctx, const MapBuf& mb) {
  const int cap = kWgThreads * ctx->wg_rows_per_thread();
  const int lim = ctx->prm.small_set_rows == 0 ? cap : std::min(ctx->prm.small_set_rows, cap);
  if (lim <= 0 || mb.nblk <= 0 || mb.max_nb > cap / kBlock) return false;
  for (int i = 0; i < ctx->n_inst; ++i)
    if (mb.cnt[i] > lim) return false;
  return true;
}

// Restricted Jacobi-PCG on H_m over the current map, starting from b in
// r[0] and x = 0 (prepared by the right-hand-side kernel).  Iterations are
// launched in budgets; after each budget the host reads the per-instance
// done flags.  Kernels of converged instances return immediately.
int run_cg(sdc_ctx* ctx, int m, const MapBuf& mb, double* x, int pred_slot, std::vector<int>* iters) {
  const int ni = ctx->n_inst;
  const Map map = mb.dev();
  const Mat H = ctx->H(m);
  const double* dinv = ctx->dinv + static_cast<int64_t>(m) * ctx->N;
  const CgStop stop = ctx->cg_stop();
  // budgets pred, pred/2, pred/4, ... (at least 2), each launched in chunks
  // that fit the event pool while kernel timing is on
  int vbudget = pred_slot >= 0 ? std::max(1, ctx->pred[pred_slot]) : 8;
  const int cap = ctx->prof && !ctx->ev.empty() ? static_cast<int>(ctx->ev.size()) / 2 : vbudget;
  int left = vbudget;
  int it = 0;
  iters->assign(ni, 0);
  if (wg_solve(ctx, mb)) {
    launch_cg_wg(ctx->stream, map, ctx->N, H, dinv, ctx->r[0], x, ctx->wg_p, stop, ctx->cg(),
                 ctx->wg_rows_per_thread());
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(ctx->h_i32, ctx->cg_done, 2 * ni * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    int mx = 0;
    for (int i = 0; i < ni; ++i) {
      const int d = ctx->h_i32[i];
      if (d == 2)
        return fail(ctx, SDC_ERR_CG_MAXIT, "CG: instance %d, node %d, sweep %d: no convergence in %d iterations",
                    i, m, ctx->k, ctx->prm.cg_maxit);
      if (d == 3)
        return fail(ctx, SDC_ERR_NONFINITE, "CG: instance %d, node %d, sweep %d: non-finite or non-positive curvature",
                    i, m, ctx->k);
      (*iters)[i] = ctx->h_i32[ni + i];
      mx = std::max(mx, (*iters)[i]);
    }
    if (pred_slot >= 0) {
      ctx->note_count(pred_slot, mx);
      ctx->pred[pred_slot] = mx + 1;
    }
    return SDC_OK;
  }
  launch_cg_start(ctx->stream, map, ni, ctx->N, H, dinv, ctx->r[0], ctx->r[1], ctx->wv[1], ctx->part[0], ctx->cg());
  HIPC(hipGetLastError());
  if (mb.nblk > 0) {
    for (;;) {
      const int budget = std::min(left, cap);
      const int it0 = it;
      const bool timed = ctx->prof && static_cast<int>(ctx->ev.size()) >= 2 * budget;
      for (int b = 0; b < budget; ++b, ++it) {
        // the start wrote the vectors to buffer 1 and the partials to buffer 0
        const int a = it & 1, o = a ^ 1;
        launch_cg_iter(ctx->stream, map, ctx->N, H, dinv, x, ctx->p, ctx->r[o], ctx->wv[o], ctx->s[o], ctx->r[a],
                       ctx->wv[a], ctx->s[a], it, ctx->part[a], ctx->part[o], ctx->cg_scal[a],
                       ctx->cg_scal[o], stop, ctx->cg(), mb.tot_if_large(ctx->cg_tot),
                       ctx->pair_all, mb.late_partials(), timed ? ctx->ev[2 * b] : nullptr,
                       timed ? ctx->ev[2 * b + 1] : nullptr);
      }
      HIPC(hipGetLastError());
      HIPC(hipMemcpyAsync(ctx->h_i32, ctx->cg_done, 2 * ni * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
      HIPC(hipStreamSynchronize(ctx->stream));
      if (timed) TRY(account_timing(ctx, mb, it0, budget, ctx->h_i32 + ni));
      bool running = false;
      for (int i = 0; i < ni; ++i) {
        const int d = ctx->h_i32[i];
        if (d == 2)
          return fail(ctx, SDC_ERR_CG_MAXIT, "CG: instance %d, node %d, sweep %d: no convergence in %d iterations",
                      i, m, ctx->k, ctx->prm.cg_maxit);
        if (d == 3)
          return fail(ctx, SDC_ERR_NONFINITE, "CG: instance %d, node %d, sweep %d: non-finite or non-positive curvature",
                      i, m, ctx->k);
        if (d == 0) running = true;
      }
      if (!running) break;
      if (it >= ctx->prm.cg_maxit + 2)
        return fail(ctx, SDC_ERR_CG_MAXIT, "CG: iteration limit reached (node %d, sweep %d)", m, ctx->k);
      left -= budget;
      if (left <= 0) {
        vbudget = std::max(2, vbudget / 2);
        left = vbudget;
      }
    }
    for (int i = 0; i < ni; ++i) (*iters)[i] = ctx->h_i32[ni + i];
  } else {
    HIPC(hipMemcpyAsync(ctx->h_i32, ctx->cg_done, ni * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
  }
  for (int i = 0; i < ni; ++i)
    if (ctx->h_i32[i] == 3)
      return fail(ctx, SDC_ERR_NONFINITE, "CG: instance %d, node %d, sweep %d: non-finite right-hand side",
                  i, m, ctx->k);
  if (pred_slot >= 0) {
    int mx = 0;
    for (int v : *iters) mx = std::max(mx, v);
    ctx->note_count(pred_slot, mx);
    ctx->pred[pred_slot] = mx + 1;
  }
  return SDC_OK;
}

// Build the work map of a device list into dyn slot `slot` (its padded copy
// in list[slot]) and fetch its sizes.
int map_list(sdc_ctx* ctx, int slot, const int32_t* idx, int64_t n) {
  MapBuf& mb = ctx->dyn[slot];
  launch_map_from_list(ctx->stream, idx, n, ctx->N, ctx->n_inst, ctx->rowptr, ctx->next(mb), ctx->list[slot]);
  HIPC(hipGetLastError());
  TRY(fetch_map(ctx, &mb));
  mb.idx = ctx->list[slot];
  return SDC_OK;
}

// Solves predicted to take more iterations than this run synchronously in
// async sweeps: a host check per budget costs little against the solve, and
// an exact count avoids redoing the step when the prediction falls short.
constexpr int kAsyncMaxBudget = 512;

// Launch node m's CG with the predicted iteration budget and no host
// synchronisation; the done flags and iteration counts are copied to the
// node's history slot on the device.  Launches after convergence return at
// once, so the result equals the synchronous path whenever the budget
// sufficed; do_sweep checks that once per sweep.
int run_cg_async(sdc_ctx* ctx, int m, const MapBuf& mb, double* x, int pred_slot, int* ev_off,
                 std::vector<int>* ev_budget) {
  const int ni = ctx->n_inst;
  const Map map = mb.dev();
  const Mat H = ctx->H(m);
  const double* dinv = ctx->dinv + static_cast<int64_t>(m) * ctx->N;
  const CgStop stop = ctx->cg_stop();
  const int p = std::max(1, ctx->pred[pred_slot]);
  const int budget = std::min(p + ctx->budget_margin(p), ctx->prm.cg_maxit + 1);
  // the kernels record the outcome straight into the node's history slot
  const CgState cg{ctx->hist_done + m * ni, ctx->hist_iters + m * ni, ctx->cg_blk_done};
  if (wg_solve(ctx, mb)) {
    launch_cg_wg(ctx->stream, map, ctx->N, H, dinv, ctx->r[0], x, ctx->wg_p, stop, cg, ctx->wg_rows_per_thread());
    HIPC(hipGetLastError());
    (*ev_budget)[m] = 0;
    return SDC_OK;
  }
  launch_cg_start(ctx->stream, map, ni, ctx->N, H, dinv, ctx->r[0], ctx->r[1], ctx->wv[1], ctx->part[0], cg);
  const bool timed = ctx->prof && static_cast<int>(ctx->ev.size()) >= 2 * (*ev_off + budget);
  for (int it = 0; mb.nblk > 0 && it < budget; ++it) {
    const int a = it & 1, o = a ^ 1;
    launch_cg_iter(ctx->stream, map, ctx->N, H, dinv, x, ctx->p, ctx->r[o], ctx->wv[o], ctx->s[o], ctx->r[a],
                   ctx->wv[a], ctx->s[a], it, ctx->part[a], ctx->part[o], ctx->cg_scal[a], ctx->cg_scal[o],
                   stop, cg, mb.tot_if_large(ctx->cg_tot), ctx->pair_all, mb.late_partials(),
                   timed ? ctx->ev[2 * (*ev_off + it)] : nullptr,
                   timed ? ctx->ev[2 * (*ev_off + it) + 1] : nullptr);
  }
  HIPC(hipGetLastError());
  (*ev_budget)[m] = timed && mb.nblk > 0 ? budget : 0;
  if (timed) *ev_off += budget;
  return SDC_OK;
}

// One sweep over the current active set; afterwards the current set is the
// one the next sweep uses (pinned, selected, or unchanged).
int do_sweep(sdc_ctx* ctx, sdc_sweep_stats* st, bool select_next, bool async,
             bool* short_budget) {
  const int M = ctx->prm.M;
  const int ni = ctx->n_inst;
  const int64_t N = ctx->N;
  const MapBuf& mb = ctx->curmap();
  const Map map = mb.dev();
  if (ctx->k < SDC_MAX_SWEEPS) {
    ctx->note_seen(ctx->k, mb.nblk);
  }
  // the statistics of this sweep refer to its own set, which the selection replaces
  std::vector<int32_t> cnt = mb.cnt;
  std::vector<int64_t> nnz = mb.nnz;
  const bool ident = mb.idx == nullptr;
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->n_active = mb.rows;
    for (int i = 0; i < ni; ++i) st->nnz_active += mb.nnz[i];
    for (auto& e : ctx->sweep_ev)
      if (!e) HIPC(hipEventCreate(&e));
    HIPC(hipEventRecord(ctx->sweep_ev[0], ctx->stream));
  }
  const EmiArgs emi = ctx->emi_args();
  const bool lin = ctx->linearized();
  launch_sweep_start(ctx->stream, M, map, N, ctx->A(), ctx->ml, ctx->v0, ctx->w0, ctx->v, ctx->w,
                     ctx->I, ctx->R, ctx->Phi, ctx->Gam, ctx->amax, ctx->cargs, emi);
  if (lin)   // this sweep's reaction Jacobian on the diagonals of H_m (rows of the map)
    launch_lin_diag(ctx->stream, M, map, N, ctx->ml, ctx->diagpos, ctx->Aval, ctx->ionic_d, ctx->v, ctx->w,
                    ctx->cargs, ctx->G, ctx->Hval, ctx->nnz, ctx->dia_H,
                    static_cast<int64_t>(ctx->nd / 2 + 1) * N, ctx->dinv);
  std::vector<std::vector<int>> iters(M);
  std::vector<int> ev_budget(M, 0);
  int ev_off = 0;
  for (int m = 0; m < M; ++m) {
    double* x = ctx->dv + m * N;
    launch_rhs(ctx->stream, M, m, map, N, ctx->A(), ctx->ml, ctx->Phi + m * N, ctx->dI, ctx->dv,
               ctx->r[0], x, ctx->cargs, emi, lin ? ctx->G : nullptr);
    HIPC(hipGetLastError());
    const int slot = ctx->pred_slot(m);
    if (async && ctx->pred[slot] <= kAsyncMaxBudget) {
      TRY(run_cg_async(ctx, m, mb, x, slot, &ev_off, &ev_budget));
    } else {
      TRY(run_cg(ctx, m, mb, x, slot, &iters[m]));
      if (async) {   // the outcome goes to the same history as an asynchronous solve's
        HIPC(hipMemcpyAsync(ctx->hist_done + m * ni, ctx->cg_done, ni * 4, hipMemcpyDeviceToDevice, ctx->stream));
        HIPC(hipMemcpyAsync(ctx->hist_iters + m * ni, ctx->cg_iters, ni * 4, hipMemcpyDeviceToDevice, ctx->stream));
      }
    }
    launch_post(ctx->stream, M, m, map, N, ctx->ionic_d, x, ctx->v + m * N, ctx->w + m * N,
                ctx->I + m * N, ctx->R + m * N, ctx->dI + m * N, ctx->dR + m * N, ctx->Gam + m * N,
                ctx->dR, ctx->amax, ctx->cargs, emi, lin);
    launch_post_sites(ctx->stream, M, m, map, N, ctx->ionic_d, ctx->v + m * N, ctx->w + m * N,
                      ctx->I + m * N, ctx->R + m * N, ctx->dI + m * N, ctx->dR + m * N, ctx->Gam + m * N,
                      ctx->dR, ctx->cargs, emi);
    if (ctx->terminate()) launch_energy(ctx->stream, map, N, ctx->H(m), x, ctx->e_part + m * ctx->all.nblk);
    HIPC(hipGetLastError());
  }
  if (lin) launch_wsweep(ctx->stream, M, map, N, ctx->ionic_d, ctx->v, ctx->w, ctx->w0, ctx->I, ctx->R, ctx->cargs);
  if (ctx->apriori_drop() && ctx->k == 0) {
    // a-priori drop tolerance of each instance for the rest of the step, from this first sweep
    launch_drop_tolerance(ctx->stream, map, M, N, ctx->ionic_d, ctx->amax, ctx->v0, ctx->w0, ctx->v, ctx->w,
                          ctx->drop_part, ctx->prm.dt, ctx->prm.rho, ctx->prm.tol_sdc, ctx->drop_theta,
                          ctx->drop_info);
    HIPC(hipGetLastError());
  }
  if (ctx->terminate()) {
    // energy-norm termination: per-instance energy and stop decision on the device
    const double q = (1.0 - ctx->prm.rho) / ctx->prm.rho * ctx->prm.tol_sdc;
    launch_energy_stop(ctx->stream, map, M, ctx->all.nblk, ctx->e_part, q * q, ctx->k + 1 >= ctx->k_min(),
                       ctx->inst_energy, ctx->inst_stop);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(ctx->h_term, ctx->inst_energy, ni * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipMemcpyAsync(reinterpret_cast<int32_t*>(ctx->h_term + ni), ctx->inst_stop, ni * 4,
                        hipMemcpyDeviceToHost, ctx->stream));
  }
  if (async) {
    // one synchronisation per sweep: the nodes' CG outcomes (and below, the next set's size)
    // (hist_iters follows hist_done in one allocation)
    HIPC(hipMemcpyAsync(ctx->h_i32 + 8 + 2 * ni, ctx->hist_done, 2 * M * ni * 4, hipMemcpyDeviceToHost,
                        ctx->stream));
  }
  if (ctx->record_dv)   // the selection below zeroes dv on the rows it drops
    HIPC(hipMemcpyAsync(ctx->record_dv, ctx->dv, static_cast<size_t>(M) * N * 8, hipMemcpyDeviceToDevice,
                        ctx->stream));
  const int next = ctx->k + 1;
  bool synced = false;
  if (next < static_cast<int>(ctx->pin.size()) && ctx->pin[next]) {
    launch_zero_rows(ctx->stream, map, ctx->zv());
    const int slot = ctx->cur == 0 ? 1 : 0;
    TRY(map_list(ctx, slot, ctx->pin[next], ctx->pin_n[next]));
    ctx->cur = slot;
    synced = true;
  } else if ((ctx->prm.theta > 0.0 || ctx->terminate() || ctx->apriori_drop()) && select_next) {
    const int slot = ctx->cur == 0 ? 1 : 0;
    MapBuf& nm = ctx->dyn[slot];
    launch_select(ctx->stream, map, ni, ctx->rowptr, ctx->amax, ctx->prm.theta,
                  ctx->apriori_drop() ? ctx->drop_theta : nullptr, ctx->sel_cnt, ctx->sel_nnz, ctx->list[slot],
                  nullptr, ctx->next(nm), ctx->zv(), ctx->terminate() ? ctx->inst_stop : nullptr);
    HIPC(hipGetLastError());
    TRY(fetch_map(ctx, &nm));
    nm.idx = ctx->list[slot];
    ctx->cur = slot;
    synced = true;
  }
  if (async) {
    if (!synced) HIPC(hipStreamSynchronize(ctx->stream));
    const int32_t* hd = ctx->h_i32 + 8 + 2 * ni;
    const int32_t* hi = hd + M * ni;
    for (int m = 0; m < M; ++m) {
      iters[m].assign(hi + m * ni, hi + (m + 1) * ni);
      int mx = 0;
      for (int i = 0; i < ni; ++i) {
        const int d = hd[m * ni + i];
        if (d == 2)
          return fail(ctx, SDC_ERR_CG_MAXIT, "CG: instance %d, node %d, sweep %d: no convergence in %d iterations",
                      i, m, ctx->k, ctx->prm.cg_maxit);
        if (d == 3)
          return fail(ctx, SDC_ERR_NONFINITE, "CG: instance %d, node %d, sweep %d: non-finite or non-positive curvature",
                      i, m, ctx->k);
        if (d == 0) {   // overran its budget: a rise beyond the margin
          if (short_budget) *short_budget = true;
          ctx->rise_now = true;
        }
        mx = std::max(mx, iters[m][i]);
      }
      const int slot = ctx->pred_slot(m);
      ctx->note_count(slot, mx);
      ctx->pred[slot] = mx + 1;
      if (ev_budget[m] > 0) {
        MapBuf view;
        view.idx = ident ? nullptr : mb.idx;
        view.cnt = cnt;
        view.nnz = nnz;
        int base = 0;
        for (int q = 0; q < m; ++q) base += ev_budget[q];
        TRY(account_timing_at(ctx, view, base, ev_budget[m], iters[m].data()));
      }
    }
  }
  if (ctx->first_subset() && ctx->k == 0) {
    // the set this step carries to the next one's first sweep: that of the
    // second sweep, or this sweep's own with one sweep per step (sdc_sweep
    // selects a next set even then; mb's slot is not the one it wrote)
    const bool own = ctx->prm.K == 1;
    const MapBuf& cm = own ? mb : ctx->curmap();
    if (own ? ident : ctx->cur < 0) {
      ctx->carry_n = -1;
    } else {
      launch_map_rows(ctx->stream, cm.dev(), ctx->carry_list);
      HIPC(hipGetLastError());
      ctx->carry_n = cm.rows;
    }
  }
  if (ctx->terminate()) {
    if (!synced && !async) HIPC(hipStreamSynchronize(ctx->stream));
    const int32_t* stop = reinterpret_cast<const int32_t*>(ctx->h_term + ni);
    ctx->all_stopped = true;
    for (int i = 0; i < ni; ++i) {
      if (st) {
        st->energy += ctx->h_term[i];
        st->n_stopped += stop[i] != 0;
      }
      ctx->all_stopped = ctx->all_stopped && stop[i] != 0;
    }
  }
  ctx->last_iters.assign(static_cast<size_t>(M) * ni, 0);
  for (int m = 0; m < M; ++m)
    for (int i = 0; i < ni && i < static_cast<int>(iters[m].size()); ++i) ctx->last_iters[m * ni + i] = iters[m][i];
  if (st) {
    for (int m = 0; m < M; ++m)
      for (int i = 0; i < ni; ++i) {
        st->cg_iters_max[m] = std::max(st->cg_iters_max[m], iters[m][i]);
        st->cg_row_iters[m] += static_cast<int64_t>(iters[m][i]) * cnt[i];
        st->cg_nnz_iters[m] += static_cast<int64_t>(iters[m][i]) * nnz[i];
      }
    st->n_next = ctx->curmap().rows;
    float ms = 0.0f;
    HIPC(hipEventRecord(ctx->sweep_ev[1], ctx->stream));
    HIPC(hipEventSynchronize(ctx->sweep_ev[1]));
    HIPC(hipEventElapsedTime(&ms, ctx->sweep_ev[0], ctx->sweep_ev[1]));
    st->ms = ms;
  }
  ctx->k = next;
  return SDC_OK;
}

// ---------------------------------------------------------------- graph-captured sweeps

// Prediction slot of node m in sweep k (steps whose first sweep takes all rows).
int pred_slot_of(const sdc_ctx* ctx, int k, int m) { return std::min(k, SDC_MAX_SWEEPS - 1) * ctx->prm.M + m; }

// CG launches captured for node m of sweep k: the predicted count (the last
// step's, plus one) and a sixteenth more, at least three (launches after
// convergence return at once).
int graph_budget(const sdc_ctx* ctx, int k, int m) {
  const int need = std::max(1, ctx->pred[pred_slot_of(ctx, k, m)]) + 1;
  return std::min(need + std::max(3, need / 16), ctx->prm.cg_maxit + 1);
}

bool graph_adaptive(const sdc_ctx* ctx) { return ctx->prm.theta > 0.0; }

// Grid of sweep k >= 1 in a graph: the map entries that sweep had in the
// last step, a quarter more and 16, at most the all-rows map's.  A set that
// outgrows it makes the step be redone (its selection covers only the grid's
// entries, so the maps built from it stay within their capacity).
int graph_cap(const sdc_ctx* ctx, int k) {
  const int seen = k < static_cast<int>(ctx->seen_nblk.size()) ? ctx->seen_nblk[k] : ctx->all.nblk;
  return std::min(ctx->all.nblk, seen + seen / 4 + 16);
}

// The map sweep k of a graph step runs on: all rows in the first sweep (and
// in every sweep without a drop tolerance), else the set the previous sweep
// selected into slot (k - 1) & 1, read through its live entry count with a
// grid of the all-rows capacity.
Map graph_map(const sdc_ctx* ctx, int k) {
  if (k == 0 || !graph_adaptive(ctx)) return ctx->all.dev();
  const int slot = (k - 1) & 1;
  const MapBuf& mb = ctx->dyn[slot];
  return Map{mb.rec, mb.inst_blk0, mb.inst_nblk, ctx->list[slot], ctx->gcap[k], ctx->n_inst, mb.totals,
             mb.xcd_shift};
}

// Enqueue sweep k of a graph step on s: the launch sequence of do_sweep with
// fixed CG budgets, each solve's outcome written to the device history of
// (k, m), and copies of that history (after the last sweep) and of the
// sweep's map sizes to pinned host memory.  Always one launch per CG
// iteration (the one-workgroup solves of small sets need the set sizes on
// the host).
int enqueue_graph_sweep(sdc_ctx* ctx, int k, hipStream_t s) {
  const int M = ctx->prm.M, K = ctx->prm.K, ni = ctx->n_inst;
  const int64_t N = ctx->N;
  const Map map = graph_map(ctx, k);
  const EmiArgs emi = ctx->emi_args();
  const CgStop stop = ctx->cg_stop();
  double* const tot = ctx->all.tot_if_large(ctx->cg_tot);
  // a listed set's instances have at most the blocks of the all-rows map's
  // instances: when those are few enough, the listed launches read their
  // partial sums themselves (as host-launched steps do, bitwise alike)
  const bool late = ctx->all.max_nb <= kTotBlocks;
  launch_sweep_start(s, M, map, N, ctx->A(), ctx->ml, ctx->v0, ctx->w0, ctx->v, ctx->w, ctx->I, ctx->R, ctx->Phi,
                     ctx->Gam, ctx->amax, ctx->cargs, emi);
  for (int m = 0; m < M; ++m) {
    double* x = ctx->dv + m * N;
    launch_rhs(s, M, m, map, N, ctx->A(), ctx->ml, ctx->Phi + m * N, ctx->dI, ctx->dv, ctx->r[0], x, ctx->cargs, emi);
    const Mat H = ctx->H(m);
    const double* dinv = ctx->dinv + static_cast<int64_t>(m) * N;
    const size_t h = (static_cast<size_t>(k) * M + m) * ni;
    const CgState cg{ctx->ghist + h, ctx->ghist + static_cast<size_t>(K) * M * ni + h, ctx->cg_blk_done};
    launch_cg_start(s, map, ni, N, H, dinv, ctx->r[0], ctx->r[1], ctx->wv[1], ctx->part[0], cg);
    const int B = ctx->gbudget[k * M + m];
    for (int it = 0; it < B; ++it) {
      const int a = it & 1, o = a ^ 1;
      launch_cg_iter(s, map, N, H, dinv, x, ctx->p, ctx->r[o], ctx->wv[o], ctx->s[o], ctx->r[a], ctx->wv[a],
                     ctx->s[a], it, ctx->part[a], ctx->part[o], ctx->cg_scal[a], ctx->cg_scal[o], stop, cg, tot,
                     ctx->pair_all, late);
    }
    launch_post(s, M, m, map, N, ctx->ionic_d, x, ctx->v + m * N, ctx->w + m * N, ctx->I + m * N, ctx->R + m * N,
                ctx->dI + m * N, ctx->dR + m * N, ctx->Gam + m * N, ctx->dR, ctx->amax, ctx->cargs, emi, false);
  }
  if (k + 1 < K && graph_adaptive(ctx)) {
    const int slot = k & 1;
    launch_select(s, map, ni, ctx->rowptr, ctx->amax, ctx->prm.theta, nullptr, ctx->sel_cnt, ctx->sel_nnz,
                  ctx->list[slot], nullptr, ctx->next(ctx->dyn[slot]), ctx->zv(), nullptr);
  }
  const size_t W = map_sizes_words(ni);
  if (k > 0 && graph_adaptive(ctx))
    HIPC(hipMemcpyAsync(ctx->gh_sizes + k * W, ctx->dyn[(k - 1) & 1].inst_nnz, W * sizeof(int64_t),
                        hipMemcpyDeviceToHost, s));
  if (k + 1 == K)
    HIPC(hipMemcpyAsync(ctx->gh_hist, ctx->ghist, 2 * static_cast<size_t>(K) * M * ni * sizeof(int32_t),
                        hipMemcpyDeviceToHost, s));
  HIPC(hipGetLastError());
  return SDC_OK;
}

void graph_release(sdc_ctx* ctx) {
  for (auto& g : ctx->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  ctx->gexec.clear();
  ctx->graph_ready = false;
}

// Capture every sweep of a step as one graph each, with the current budgets.
int graph_capture(sdc_ctx* ctx) {
  const int K = ctx->prm.K, M = ctx->prm.M;
  graph_release(ctx);
  ctx->gexec.assign(K, nullptr);
  ctx->gbudget.assign(static_cast<size_t>(K) * M, 0);
  ctx->gcap.assign(K, ctx->all.nblk);
  for (int k = 0; k < K; ++k) {
    for (int m = 0; m < M; ++m) ctx->gbudget[k * M + m] = graph_budget(ctx, k, m);
    if (k > 0) ctx->gcap[k] = graph_cap(ctx, k);
  }
  for (int k = 0; k < K; ++k) {
    HIPC(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_graph_sweep(ctx, k, ctx->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (rc != SDC_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      graph_release(ctx);
      return rc != SDC_OK ? rc : fail(ctx, SDC_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(&ctx->gexec[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      graph_release(ctx);
      return fail(ctx, SDC_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
  }
  ctx->graph_ready = true;
  ++ctx->graph_captures;
  return SDC_OK;
}

// The sweeps of a started step as K graph launches and one synchronisation.
// Re-captures first when a predicted CG count no longer fits its budget, a
// set of the last step, grown once more by twice its last growth, would
// exceed its grid (growing fronts: captured again before the set outgrows
// it, which would redo the step) or a grid is twice what the last step
// needed; sets
// *short_budget (and changes nothing the caller keeps) when a solve did not
// finish within its budget or a set outgrew its grid, so that the caller
// redoes the step.
int graph_step(sdc_ctx* ctx, sdc_step_stats* st, bool* short_budget) {
  const int K = ctx->prm.K, M = ctx->prm.M, ni = ctx->n_inst;
  bool fits = ctx->graph_ready;
  for (int k = 0; fits && k < K; ++k) {
    for (int m = 0; m < M; ++m)
      if (std::max(1, ctx->pred[pred_slot_of(ctx, k, m)]) + 1 > ctx->gbudget[k * M + m]) fits = false;
    if (k > 0 && graph_adaptive(ctx)) {
      const int seen = k < static_cast<int>(ctx->seen_nblk.size()) ? ctx->seen_nblk[k] : ctx->all.nblk;
      const int prev = k < static_cast<int>(ctx->seen_prev.size()) ? ctx->seen_prev[k] : seen;
      // the set may grow within this step as much as twice its last growth
      if (seen + 2 * std::max(0, seen - prev) > ctx->gcap[k] || ctx->gcap[k] > 2 * graph_cap(ctx, k)) fits = false;
    }
  }
  if (!fits) TRY(graph_capture(ctx));
  HIPC(hipEventRecord(ctx->gev[0], ctx->stream));
  for (int k = 0; k < K; ++k) {
    HIPC(hipGraphLaunch(ctx->gexec[k], ctx->stream));
    HIPC(hipEventRecord(ctx->gev[k + 1], ctx->stream));
  }
  HIPC(hipStreamSynchronize(ctx->stream));
  ++ctx->graph_steps;
  // a set that outgrew its sweep's grid: that sweep and the ones after it
  // worked on part of their sets, so their outcome means nothing; redo
  const size_t W = map_sizes_words(ni);
  ctx->seen_nblk.resize(K, ctx->all.nblk);
  for (int k = 1; k < K && graph_adaptive(ctx); ++k) {
    const int32_t* tot = reinterpret_cast<const int32_t*>(ctx->gh_sizes + k * W + ni + 1);
    ctx->note_seen(k, tot[0]);
    if (tot[0] > ctx->gcap[k] || tot[2] != 0) *short_budget = true;
  }
  if (*short_budget) return SDC_OK;
  const int32_t* done = ctx->gh_hist;
  const int32_t* iters = ctx->gh_hist + static_cast<size_t>(K) * M * ni;
  for (int k = 0; k < K; ++k)
    for (int m = 0; m < M; ++m)
      for (int i = 0; i < ni; ++i) {
        const int d = done[(k * M + m) * ni + i];
        if (d == 2)
          return fail(ctx, SDC_ERR_CG_MAXIT, "CG: instance %d, node %d, sweep %d: no convergence in %d iterations",
                      i, m, k, ctx->prm.cg_maxit);
        if (d == 3)
          return fail(ctx, SDC_ERR_NONFINITE, "CG: instance %d, node %d, sweep %d: non-finite or non-positive "
                      "curvature", i, m, k);
        if (d == 0) *short_budget = true;
      }
  if (*short_budget) return SDC_OK;
  // the outcome: predictions, the last sweep's counts, the host mirror of the maps
  if (st) std::memset(st, 0, sizeof *st);
  for (int k = 0; k < K; ++k) {
    const MapBuf* mb = &ctx->all;
    if (k > 0 && graph_adaptive(ctx)) {
      const int slot = (k - 1) & 1;
      mb = &ctx->dyn[slot];
      TRY(parse_map_sizes(ctx, &ctx->dyn[slot], ctx->gh_sizes + k * W));
      ctx->dyn[slot].idx = ctx->list[slot];
    }
    for (int m = 0; m < M; ++m) {
      int mx = 0;
      for (int i = 0; i < ni; ++i) mx = std::max(mx, iters[(k * M + m) * ni + i]);
      ctx->note_count(pred_slot_of(ctx, k, m), mx);
      ctx->pred[pred_slot_of(ctx, k, m)] = mx + 1;
    }
    if (st) {
      sdc_sweep_stats& q = st->sweep[k];
      q.n_active = mb->rows;
      for (int i = 0; i < ni; ++i) q.nnz_active += mb->nnz[i];
      for (int m = 0; m < M; ++m)
        for (int i = 0; i < ni; ++i) {
          const int it = iters[(k * M + m) * ni + i];
          q.cg_iters_max[m] = std::max(q.cg_iters_max[m], it);
          q.cg_row_iters[m] += static_cast<int64_t>(it) * mb->cnt[i];
          q.cg_nnz_iters[m] += static_cast<int64_t>(it) * mb->nnz[i];
        }
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, ctx->gev[k], ctx->gev[k + 1]));
      q.ms = ms;
      if (k > 0) st->sweep[k - 1].n_next = q.n_active;
    }
  }
  if (st) {
    st->n_sweeps = K;
    st->sweep[K - 1].n_next = st->sweep[K - 1].n_active;
  }
  ctx->last_iters.assign(iters + static_cast<size_t>(K - 1) * M * ni, iters + static_cast<size_t>(K) * M * ni);
  ctx->cur = K >= 2 && graph_adaptive(ctx) ? (K - 2) & 1 : -1;
  ctx->k = K;
  return SDC_OK;
}

// Diagonal storage: per instance, the distinct column offsets (col - row) of
// its rows, sorted; usable when every instance has the same number nd <=
// kMaxDiag of them, as a set symmetric about 0 (a symmetric pattern).  Since
// A and H_m are symmetric, only the nd/2 + 1 diagonals with offset >= 0 are
// stored: entry (r, r + o), o >= 0, at dval[o's index][r], and (r, r - o) is
// read as (r - o, r).  Entries absent from the pattern hold 0.
int build_dia(sdc_ctx* ctx) {
  if (ctx->emi) return SDC_OK;   // the membrane partner columns do not form diagonals
  const int ni = ctx->n_inst;
  const int64_t N = ctx->N;
  const HostSystem& hs = ctx->host;
  std::vector<std::vector<int32_t>> offs(ni);
  for (int i = 0; i < ni; ++i) {
    std::vector<int32_t> o;
    for (int64_t r = ctx->node_off_h[i]; r < ctx->node_off_h[i + 1]; ++r)
      for (int32_t e = hs.rowptr[r]; e < hs.rowptr[r + 1]; ++e) {
        const int32_t d = hs.col[e] - static_cast<int32_t>(r);
        if (std::find(o.begin(), o.end(), d) == o.end()) {
          o.push_back(d);
          if (static_cast<int>(o.size()) > kMaxDiag) return SDC_OK;   // not diagonal-structured
        }
      }
    std::sort(o.begin(), o.end());
    offs[i] = std::move(o);
  }
  const int nd = static_cast<int>(offs[0].size());
  for (int i = 0; i < ni; ++i) {
    if (static_cast<int>(offs[i].size()) != nd) return SDC_OK;
    for (int d = 0; d < nd; ++d)
      if (offs[i][d] != -offs[i][nd - 1 - d]) return SDC_OK;
  }
  const int h = nd / 2;   // index of offset 0
  std::vector<int32_t> off(static_cast<size_t>(ni) * nd, 0);
  for (int i = 0; i < ni; ++i)
    for (int d = 0; d < nd; ++d) off[i * nd + d] = offs[i][d];
  const int ns = h + 1;   // stored diagonals
  std::vector<double> val(static_cast<size_t>(ns) * N, 0.0);
  for (int i = 0; i < ni; ++i)
    for (int64_t r = ctx->node_off_h[i]; r < ctx->node_off_h[i + 1]; ++r)
      for (int32_t e = hs.rowptr[r]; e < hs.rowptr[r + 1]; ++e) {
        const int32_t d = hs.col[e] - static_cast<int32_t>(r);
        if (d < 0) continue;
        const auto& o = offs[i];
        const int q = static_cast<int>(std::lower_bound(o.begin(), o.end(), d) - o.begin());
        val[static_cast<size_t>(q - h) * N + r] = hs.val[e];
      }
  const int M = ctx->prm.M;
  if (!ctx->dia_off) {
    TRY(dalloc(ctx, &ctx->dia_off, off.size()));
    TRY(dalloc(ctx, &ctx->dia_A, val.size()));
    TRY(dalloc(ctx, &ctx->dia_H, val.size() * M));
  }
  HIPC(hipMemcpyAsync(ctx->dia_off, off.data(), off.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  ctx->dia_off_h = off;
  HIPC(hipMemcpyAsync(ctx->dia_A, val.data(), val.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  for (int m = 0; m < M; ++m)
    launch_build_h_dia(ctx->stream, N, 0, static_cast<int>(N), ns, ctx->dia_A, ctx->ml,
                       ctx->prm.dt * ctx->col.QI[m][m], ctx->dia_H + static_cast<int64_t>(m) * ns * N);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(ctx->stream));   // the host staging vector goes out of scope
  ctx->nd = nd;
  return SDC_OK;
}

// The sliced ELL values of A and every H_m from their CSR values.
int fill_sell(sdc_ctx* ctx) {
  if (!ctx->sell_ptr) return SDC_OK;
  launch_build_sell(ctx->stream, ctx->N, ctx->nslice, ctx->rowptr, ctx->sell_ptr, ctx->Aval, ctx->sell_A);
  for (int m = 0; m < ctx->prm.M; ++m)
    launch_build_sell(ctx->stream, ctx->N, ctx->nslice, ctx->rowptr, ctx->sell_ptr, ctx->Hval + m * ctx->nnz,
                      ctx->sell_H + m * ctx->sell_len);
  HIPC(hipGetLastError());
  return SDC_OK;
}

// Sliced ELL copy (format 3, and a candidate of the timed choice): slices of
// kSlice consecutive rows, each padded to its longest row, entries column by
// column; columns built on the host, values copied on the device from the
// CSR values of A and every H_m (bitwise the same entries).
int build_sell(sdc_ctx* ctx) {
  const int64_t N = ctx->N;
  const HostSystem& hs = ctx->host;
  const int ns = static_cast<int>((N + kSlice - 1) / kSlice);
  std::vector<int32_t> ptr(ns + 1, 0);
  for (int sl = 0; sl < ns; ++sl) {
    int len = 0;
    for (int64_t r = static_cast<int64_t>(sl) * kSlice; r < std::min<int64_t>(N, (sl + 1) * int64_t(kSlice)); ++r)
      len = std::max(len, hs.rowptr[r + 1] - hs.rowptr[r]);
    const int64_t next = static_cast<int64_t>(ptr[sl]) + static_cast<int64_t>(len) * kSlice;
    if (next >= (int64_t(1) << 31)) return SDC_OK;   // too large for int32 offsets: no copy
    ptr[sl + 1] = static_cast<int32_t>(next);
  }
  const int64_t len_all = ptr[ns];
  std::vector<int32_t> col(static_cast<size_t>(len_all), 0);
  for (int sl = 0; sl < ns; ++sl) {
    const int len = (ptr[sl + 1] - ptr[sl]) / kSlice;
    for (int lane = 0; lane < kSlice; ++lane) {
      const int64_t r = static_cast<int64_t>(sl) * kSlice + lane;
      for (int d = 0; d < len; ++d) {
        int32_t c = 0;
        if (r < N) c = d < hs.rowptr[r + 1] - hs.rowptr[r] ? hs.col[hs.rowptr[r] + d] : static_cast<int32_t>(r);
        col[static_cast<size_t>(ptr[sl]) + static_cast<size_t>(d) * kSlice + lane] = c;
      }
    }
  }
  const int M = ctx->prm.M;
  TRY(dalloc(ctx, &ctx->sell_ptr, ns + 1));
  TRY(dalloc(ctx, &ctx->sell_col, len_all));
  TRY(dalloc(ctx, &ctx->sell_A, len_all));
  TRY(dalloc(ctx, &ctx->sell_H, static_cast<size_t>(M) * len_all));
  HIPC(hipMemcpyAsync(ctx->sell_ptr, ptr.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->sell_col, col.data(), len_all * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  ctx->nslice = ns;
  ctx->sell_len = len_all;
  TRY(fill_sell(ctx));
  HIPC(hipStreamSynchronize(ctx->stream));   // the host staging vectors go out of scope
  return SDC_OK;
}

// Storage choice (unless the caller forced one): the diagonal copy when it
// reads at most 0.6 of CSR's matrix bytes (8 B per stored diagonal and row
// against 12 B per entry with its column index: 2D triangles 0.38, 3D
// tetrahedra 0.52); otherwise time the CG start kernel (an SpMV with H_0
// over all rows) in both storages and keep the diagonal copy unless CSR is
// faster by more than 5 %.  On small systems both times are launch
// overhead, and a profiler's per-dispatch cost can invert them by chance;
// the timings are taken and reported either way.
int autotune(sdc_ctx* ctx) {
  ctx->use_dia = false;
  ctx->use_sell = false;
  if (ctx->prm.format == 1) return SDC_OK;
  if (ctx->prm.format == 2) {
    ctx->use_dia = true;
    return SDC_OK;
  }
  if (ctx->prm.format == 3) {
    ctx->use_sell = true;
    return SDC_OK;
  }
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  const Map map = ctx->all.dev();
  // interleaved rounds, keep each storage's fastest round (robust to noise);
  // candidates: CSR, the diagonal copy, the sliced ELL copy (those built)
  double t[3] = {1e30, 1e30, 1e30};
  const bool cand[3] = {true, ctx->nd > 0, ctx->sell_ptr != nullptr};
  const int reps = 10;
  for (int round = 0; round < 4; ++round)
    for (int f = 0; f < 3; ++f) {
      if (!cand[f]) continue;
      const Mat H = ctx->matH(0, f + 1);
      launch_cg_start(ctx->stream, map, ctx->n_inst, ctx->N, H, ctx->dinv, ctx->r[0], ctx->r[1], ctx->wv[1],
                      ctx->part[0], ctx->cg());
      HIPC(hipEventRecord(e0, ctx->stream));
      for (int rep = 0; rep < reps; ++rep)
        launch_cg_start(ctx->stream, map, ctx->n_inst, ctx->N, H, ctx->dinv, ctx->r[0], ctx->r[1], ctx->wv[1],
                        ctx->part[0], ctx->cg());
      HIPC(hipEventRecord(e1, ctx->stream));
      HIPC(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, e0, e1));
      t[f] = std::min(t[f], 1e3 * ms / reps);
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->t_csr_us = t[0];
  ctx->t_dia_us = cand[1] ? t[1] : 0.0;
  ctx->t_sell_us = cand[2] ? t[2] : 0.0;
  if (cand[1]) {
    const double dia_bytes = 8.0 * (ctx->nd / 2 + 1) * static_cast<double>(ctx->N);
    const double csr_bytes = 12.0 * static_cast<double>(ctx->nnz);
    ctx->use_dia = dia_bytes <= 0.6 * csr_bytes || t[1] < 1.05 * std::min(t[0], t[2]);
  }
  // the sliced ELL copy when it beats CSR by 3 % (and the diagonal copy is not kept)
  ctx->use_sell = !ctx->use_dia && cand[2] && t[2] < 0.97 * t[0];
  return SDC_OK;
}

// Rows per thread of the CG launches over all rows with diagonal storage
// (rows_per_thread 0): a CG started from b = ML on all rows, its first
// iteration, then alternating rounds of its second iteration with one and
// with two rows per thread.  That launch reads one parity of the buffers and
// writes the other (x and p in place), so every repetition has the same
// inputs and the same work; the fastest round of each counts, and two rows
// stay unless one row is faster by 3 %.  The work buffers are cleared after.
// Maps under kTuneMinBlocks keep two rows untimed: such launches are
// latency-bound, the two variants time alike within noise, and a timed
// choice there would only make otherwise identical runs differ.
constexpr int kTuneMinBlocks = 2048;

int tune_rows_per_thread(sdc_ctx* ctx) {
  ctx->pair_all = ctx->prm.rows_per_thread != 1;
  if (!ctx->use_dia || ctx->prm.rows_per_thread != 0 || !compiled_diagonals(ctx->nd) ||
      ctx->all.nblk < kTuneMinBlocks)
    return SDC_OK;
  const Map map = ctx->all.dev();
  const Mat H = ctx->H(0);
  const int64_t N = ctx->N;
  double* const tot = ctx->all.tot_if_large(ctx->cg_tot);
  const auto iterate = [&](int it, bool pair) {
    const int a = it & 1, o = a ^ 1;
    launch_cg_iter(ctx->stream, map, N, H, ctx->dinv, ctx->dv, ctx->p, ctx->r[o], ctx->wv[o], ctx->s[o], ctx->r[a],
                   ctx->wv[a], ctx->s[a], it, ctx->part[a], ctx->part[o], ctx->cg_scal[a], ctx->cg_scal[o],
                   CgStop{0.0, 0.0, ctx->prm.cg_maxit + 2, 0}, ctx->cg(), tot, pair);
  };
  launch_copy_b(ctx->stream, map, ctx->ml, ctx->r[0], ctx->dv);
  launch_cg_start(ctx->stream, map, ctx->n_inst, N, H, ctx->dinv, ctx->r[0], ctx->r[1], ctx->wv[1], ctx->part[0],
                  ctx->cg());
  iterate(0, true);
  HIPC(hipGetLastError());
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  double t[2] = {1e30, 1e30};   // one row, two rows per thread
  const int reps = 10;
  for (int round = 0; round < 4; ++round)
    for (int v = 0; v < 2; ++v) {
      iterate(1, v == 1);
      HIPC(hipEventRecord(e0, ctx->stream));
      for (int rep = 0; rep < reps; ++rep) iterate(1, v == 1);
      HIPC(hipEventRecord(e1, ctx->stream));
      HIPC(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPC(hipEventElapsedTime(&ms, e0, e1));
      t[v] = std::min(t[v], 1e3 * ms / reps);
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPC(hipGetLastError());
  ctx->t_rows_us[0] = t[0];
  ctx->t_rows_us[1] = t[1];
  ctx->pair_all = !(t[0] < 0.97 * t[1]);
  // back to the state a new context has
  for (int q = 0; q < 2; ++q) {
    for (double* b : {ctx->r[q], ctx->wv[q], ctx->s[q]}) HIPC(hipMemsetAsync(b, 0, N * 8, ctx->stream));
    HIPC(hipMemsetAsync(ctx->part[q], 0, 4 * sizeof(double) * ctx->all.nblk, ctx->stream));
    HIPC(hipMemsetAsync(ctx->cg_scal[q], 0, kScal * sizeof(double) * ctx->n_inst, ctx->stream));
  }
  HIPC(hipMemsetAsync(ctx->p, 0, N * 8, ctx->stream));
  HIPC(hipMemsetAsync(ctx->dv, 0, static_cast<size_t>(ctx->prm.M) * N * 8, ctx->stream));
  HIPC(hipMemsetAsync(ctx->cg_done, 0, 2 * ctx->n_inst * sizeof(int32_t), ctx->stream));
  HIPC(hipMemsetAsync(ctx->cg_blk_done, 0, ctx->all.nblk * sizeof(int32_t), ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  return SDC_OK;
}

// The rows of the first sweep of the step starting at t (first_rings > 0):
// all rows (first_n = -1) on the first step, on every first_full_every-th
// and when nothing is carried; else the carried rows and this step's
// stimulated rows, grown first_rings times by their mesh neighbours,
// compacted into first_list.
int build_first_set(sdc_ctx* ctx, double t) {
  ctx->first_n = -1;
  if (!ctx->first_subset()) return SDC_OK;
  const int64_t step = ctx->step_count++;
  const int F = ctx->prm.first_full_every;
  if (ctx->carry_n < 0 || (F <= 0 ? step == 0 : step % F == 0)) return SDC_OK;
  const int64_t N = ctx->N;
  launch_mark_clear(ctx->stream, ctx->mark[0], N);
  launch_mark_rows(ctx->stream, ctx->carry_list, ctx->carry_n, ctx->mark[0]);
  for (const auto& s : ctx->stims)
    if (stimulus_applies(s, t, ctx->prm.dt)) launch_mark_rows(ctx->stream, s.nodes, s.n, ctx->mark[0]);
  int a = 0;
  for (int r = 0; r < ctx->prm.first_rings; ++r, a ^= 1)
    launch_mark_grow(ctx->stream, ctx->rowptr, ctx->colidx, ctx->mark[a], ctx->mark[a ^ 1], N);
  HIPC(hipGetLastError());
  // the marked rows, in order: a selection over all rows with threshold 1/2
  MapBuf& nm = ctx->dyn[0];
  launch_select(ctx->stream, ctx->all.dev(), ctx->n_inst, ctx->rowptr, ctx->mark[a], 0.5, nullptr, ctx->sel_cnt,
                ctx->sel_nnz, ctx->list[0], ctx->first_list, ctx->next(nm), ctx->zv(), nullptr);
  HIPC(hipGetLastError());
  TRY(fetch_map(ctx, &nm));
  ctx->first_n = nm.rows;
  return SDC_OK;
}

// Spread the saved start state (v0, w0) to all nodes; all rows active (or
// the step's heuristic first-sweep set).
int restart_step(sdc_ctx* ctx) {
  launch_spread(ctx->stream, ctx->prm.M, ctx->all.dev(), ctx->N, ctx->ionic_d, ctx->v0, ctx->w0, ctx->v,
                ctx->w, ctx->I, ctx->R, ctx->emi_args());
  HIPC(hipGetLastError());
  ctx->cur = -1;
  ctx->k = 0;
  ctx->in_step = true;
  if (ctx->first_n >= 0) {
    // a heuristic first-sweep set: the vectors read at neighbouring columns
    // start at zero off it
    launch_zero_rows(ctx->stream, ctx->all.dev(), ctx->zv());
    HIPC(hipGetLastError());
    TRY(map_list(ctx, 0, ctx->first_list, ctx->first_n));
    ctx->cur = 0;
  }
  if (ctx->terminate()) {
    HIPC(hipMemsetAsync(ctx->inst_stop, 0, ctx->n_inst * 4, ctx->stream));
    ctx->all_stopped = false;
  }
  return SDC_OK;
}

// Cell-by-cell model, host part of the setup: validate the couplings, merge
// the gap junctions, the membrane pairs (pattern only) and the Robin term
// into A, and form the membrane mass and the per-node site arrays.
int emi_host_setup(sdc_ctx* ctx, const sdc_emi* emi, std::vector<int32_t>* part, std::vector<double>* sl,
                   std::vector<int32_t>* ppos, std::vector<double>* pmass) {
  const int64_t N = ctx->N;
  if (ctx->n_inst != 1) return fail(ctx, SDC_ERR_ARG, "the cell-by-cell model takes one instance");
  if (ctx->prm.format == 2) return fail(ctx, SDC_ERR_ARG, "the cell-by-cell model uses CSR storage");
  if (emi->n_mem < 0 || emi->n_gap < 0 || !(emi->cm > 0.0) || !(emi->eps >= 0.0) || !(emi->g_gap >= 0.0) ||
      !emi->robin_len || (emi->n_mem > 0 && (!emi->mem_intra || !emi->mem_extra || !emi->mem_len)) ||
      (emi->n_gap > 0 && (!emi->gap_a || !emi->gap_b || !emi->gap_len)))
    return fail(ctx, SDC_ERR_ARG, "bad cell-by-cell description");
  part->assign(N, -1);
  sl->assign(N, 0.0);
  for (int64_t q = 0; q < emi->n_mem; ++q) {
    const int32_t i = emi->mem_intra[q], x = emi->mem_extra[q];
    if (i < 0 || i >= N || x < 0 || x >= N || i == x || !(emi->mem_len[q] > 0.0))
      return fail(ctx, SDC_ERR_ARG, "membrane site %lld: bad nodes or length", static_cast<long long>(q));
    if ((*part)[i] >= 0 || (*part)[x] >= 0)
      return fail(ctx, SDC_ERR_ARG, "membrane site %lld: node already in a site", static_cast<long long>(q));
    (*part)[i] = x;
    (*part)[x] = i;
    (*sl)[i] = emi->mem_len[q];
    (*sl)[x] = -emi->mem_len[q];
  }
  for (int64_t q = 0; q < N; ++q)
    if (!(emi->robin_len[q] >= 0.0)) return fail(ctx, SDC_ERR_ARG, "negative Robin length");
  const int64_t np = emi->n_gap + emi->n_mem;
  std::vector<int32_t> a(np), b(np);
  std::vector<double> w(np, 0.0), robin(N);
  for (int64_t q = 0; q < emi->n_gap; ++q) {
    a[q] = emi->gap_a[q];
    b[q] = emi->gap_b[q];
    w[q] = emi->g_gap * emi->gap_len[q];
  }
  for (int64_t q = 0; q < emi->n_mem; ++q) {
    a[emi->n_gap + q] = emi->mem_intra[q];
    b[emi->n_gap + q] = emi->mem_extra[q];
  }
  for (int64_t q = 0; q < N; ++q) robin[q] = emi->eps * emi->robin_len[q];
  std::string e = add_pair_couplings(&ctx->host, np, a.data(), b.data(), w.data(), robin.data());
  if (!e.empty()) return fail(ctx, SDC_ERR_ARG, "cell-by-cell couplings: %s", e.c_str());
  HostSystem& hs = ctx->host;
  ppos->assign(N, -1);
  pmass->assign(N, 0.0);
  for (int64_t r = 0; r < N; ++r) {
    hs.ml[r] = emi->cm * std::fabs((*sl)[r]);
    if ((*part)[r] < 0) continue;
    const int32_t* rc = hs.col.data() + hs.rowptr[r];
    const int32_t len = hs.rowptr[r + 1] - hs.rowptr[r];
    (*ppos)[r] = static_cast<int32_t>(std::lower_bound(rc, rc + len, (*part)[r]) - rc) + hs.rowptr[r];
    (*pmass)[r] = -emi->cm * std::fabs((*sl)[r]);
  }
  return SDC_OK;
}

int check_ready(sdc_ctx* ctx) {
  if (!ctx) return SDC_ERR_ARG;
  if (!ctx->ready) return fail(ctx, SDC_ERR_STATE, "sdc_setup_mesh has not been called");
  HIPC(hipSetDevice(ctx->device));
  return SDC_OK;
}

}  // namespace sdc

// ---------------------------------------------------------------- ABI

extern "C" {

int sdc_create(sdc_ctx** out, int32_t device, void* stream) {
  if (!out) return SDC_ERR_ARG;
  *out = nullptr;
  sdc_ctx* ctx = new (std::nothrow) sdc_ctx();
  if (!ctx) return SDC_ERR_OOM;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(stream);
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    delete ctx;
    return SDC_ERR_HIP;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return SDC_ERR_HIP;
  }
  *out = ctx;
  return SDC_OK;
}

void sdc_destroy(sdc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (auto& s : ctx->stims) (void)hipFree(s.nodes);
  for (auto* p : ctx->pin) if (p) (void)hipFree(p);
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  for (auto e : ctx->sweep_ev) if (e) (void)hipEventDestroy(e);
  graph_release(ctx);
  for (auto e : ctx->gev) if (e) (void)hipEventDestroy(e);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->gh_hist) (void)hipHostFree(ctx->gh_hist);
  if (ctx->gh_sizes) (void)hipHostFree(ctx->gh_sizes);
  if (ctx->h_i32) (void)hipHostFree(ctx->h_i32);
  if (ctx->h_i64) (void)hipHostFree(ctx->h_i64);
  if (ctx->h_term) (void)hipHostFree(ctx->h_term);
  delete ctx;
}

const char* sdc_last_error(const sdc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sdc_set_stream(sdc_ctx* ctx, void* stream) {
  if (!ctx) return SDC_ERR_ARG;
  ctx->stream = static_cast<hipStream_t>(stream);
  return SDC_OK;
}

int sdc_collocation(int32_t M, double* tau, double* Q, double* QI, double* QE) {
  Collocation c;
  if (M < 1 || M > SDC_MAX_NODES || collocation(M, &c) != 0) return SDC_ERR_ARG;
  for (int m = 0; m < M; ++m) {
    if (tau) tau[m] = c.tau[m];
    for (int j = 0; j < M; ++j) {
      if (Q) Q[m * M + j] = c.Q[m][j];
      if (QI) QI[m * M + j] = c.QI[m][j];
      if (QE) QE[m * M + j] = c.QE[m][j];
    }
  }
  return SDC_OK;
}

int sdc_setup_mesh(sdc_ctx* ctx, const sdc_params* prm, int32_t dim, int32_t n_inst,
                   const int64_t* node_off, const double* coords, const int64_t* elem_off,
                   const int32_t* elems, const double* elem_tensor, const double* node_sigma,
                   const double* ionic, const sdc_emi* emi) {
  if (!ctx) return SDC_ERR_ARG;
  if (ctx->ready) return fail(ctx, SDC_ERR_STATE, "sdc_setup_mesh may be called once per context");
  if (!prm || !node_off || !coords || !elem_off || !elems || !elem_tensor || !node_sigma || !ionic)
    return fail(ctx, SDC_ERR_ARG, "null argument");
  if (prm->M < 1 || prm->M > SDC_MAX_NODES) return fail(ctx, SDC_ERR_ARG, "M must be in 1..%d", SDC_MAX_NODES);
  if (prm->K < 1 || prm->K > SDC_MAX_SWEEPS) return fail(ctx, SDC_ERR_ARG, "K must be in 1..%d", SDC_MAX_SWEEPS);
  if (!(prm->dt > 0.0) || !(prm->cg_rtol > 0.0) || prm->cg_maxit < 1 || prm->format < 0 || prm->format > 3)
    return fail(ctx, SDC_ERR_ARG, "dt, cg_rtol must be > 0, cg_maxit >= 1, format in 0..3");
  if (prm->tol_sdc > 0.0 && !(prm->rho > 0.0 && prm->rho < 1.0))
    return fail(ctx, SDC_ERR_ARG, "energy-norm termination needs 0 < rho < 1");
  if (prm->drop_mode < 0 || prm->drop_mode > 1) return fail(ctx, SDC_ERR_ARG, "drop_mode must be 0 or 1");
  if (prm->drop_mode == 1 && !(prm->tol_sdc > 0.0))
    return fail(ctx, SDC_ERR_ARG, "the a-priori drop tolerance needs tol_sdc > 0 (and 0 < rho < 1)");
  if (prm->drop_mode == 1 && emi)
    return fail(ctx, SDC_ERR_ARG, "the a-priori drop tolerance is defined for the monodomain model only");
  if (prm->scheme < 0 || prm->scheme > 1) return fail(ctx, SDC_ERR_ARG, "scheme must be 0 or 1");
  if (prm->scheme == 1 && emi)
    return fail(ctx, SDC_ERR_ARG, "the linearized scheme is implemented for the monodomain model only");
  if (prm->first_rings < 0) return fail(ctx, SDC_ERR_ARG, "first_rings must be >= 0");
  if (prm->small_set_rows < -1) return fail(ctx, SDC_ERR_ARG, "small_set_rows must be >= -1");
  if (prm->rows_per_thread < 0 || prm->rows_per_thread > 2)
    return fail(ctx, SDC_ERR_ARG, "rows_per_thread must be 0, 1 or 2");
  if (prm->first_rings > 0 && emi)
    return fail(ctx, SDC_ERR_ARG, "the heuristic first-sweep set is implemented for the monodomain model only");
  if (!(prm->cg_energy_tol >= 0.0) || !std::isfinite(prm->cg_energy_tol))
    return fail(ctx, SDC_ERR_ARG, "cg_energy_tol must be finite and >= 0");
  if (prm->cg_energy_tol > 0.0 && (prm->cg_delay < 1 || prm->cg_delay > kMaxDelay))
    return fail(ctx, SDC_ERR_ARG, "the energy-error stop needs cg_delay in 1..%d", kMaxDelay);
  if (prm->cg_energy_tol > 0.0 && emi)
    return fail(ctx, SDC_ERR_ARG, "the energy-error CG stop is implemented for the monodomain model only");
  if (dim < 1 || dim > 3 || n_inst < 1) return fail(ctx, SDC_ERR_ARG, "dim in 1..3 and n_inst >= 1 required");
  if (node_off[0] != 0 || elem_off[0] != 0) return fail(ctx, SDC_ERR_ARG, "offsets must start at 0");
  for (int i = 0; i < n_inst; ++i)
    if (node_off[i + 1] <= node_off[i] || elem_off[i + 1] < elem_off[i])
      return fail(ctx, SDC_ERR_ARG, "instance %d: empty or decreasing offsets", i);
  const int64_t N = node_off[n_inst], E = elem_off[n_inst];
  if (N >= (int64_t(1) << 31) - kBlock) return fail(ctx, SDC_ERR_ARG, "too many nodes");
  const int nv = dim + 1;
  for (int i = 0; i < n_inst; ++i)
    for (int64_t e = elem_off[i]; e < elem_off[i + 1]; ++e)
      for (int a = 0; a < nv; ++a) {
        const int64_t g = elems[e * nv + a];
        if (g < node_off[i] || g >= node_off[i + 1])
          return fail(ctx, SDC_ERR_ARG, "element %lld of instance %d uses node %lld outside it",
                      static_cast<long long>(e), i, static_cast<long long>(g));
      }
  HIPC(hipSetDevice(ctx->device));
  ctx->prm = *prm;
  if (collocation(prm->M, &ctx->col) != 0) return fail(ctx, SDC_ERR_ARG, "collocation setup failed");
  std::memset(&ctx->cargs, 0, sizeof ctx->cargs);
  for (int m = 0; m < prm->M; ++m)
    for (int j = 0; j < prm->M; ++j) {
      ctx->cargs.Q[m][j] = ctx->col.Q[m][j];
      ctx->cargs.QI[m][j] = ctx->col.QI[m][j];
      ctx->cargs.QE[m][j] = ctx->col.QE[m][j];
    }
  ctx->cargs.dt = prm->dt;
  ctx->dim = dim;
  ctx->n_inst = n_inst;
  ctx->N = N;
  ctx->node_off_h.assign(node_off, node_off + n_inst + 1);

  std::string e = assemble_p1(dim, N, coords, E, elems, elem_tensor, node_sigma, &ctx->host);
  if (!e.empty()) return fail(ctx, SDC_ERR_ARG, "assembly: %s", e.c_str());
  std::vector<int32_t> emi_part, emi_ppos;
  std::vector<double> emi_sl, emi_pmass;
  if (emi) TRY(emi_host_setup(ctx, emi, &emi_part, &emi_sl, &emi_ppos, &emi_pmass));
  ctx->nnz = ctx->host.rowptr[N];
  for (int64_t i = 0; i < N; ++i)
    ctx->max_row = std::max<int64_t>(ctx->max_row, ctx->host.rowptr[i + 1] - ctx->host.rowptr[i]);
  const int64_t nnz = ctx->nnz;
  const int M = prm->M;

  TRY(dalloc(ctx, &ctx->rowptr, N + 1));
  TRY(dalloc(ctx, &ctx->colidx, nnz));
  TRY(dalloc(ctx, &ctx->diagpos, N));
  TRY(dalloc(ctx, &ctx->Aval, nnz));
  TRY(dalloc(ctx, &ctx->Hval, nnz * M));
  TRY(dalloc(ctx, &ctx->ml, N));
  TRY(dalloc(ctx, &ctx->dinv, N * M));
  TRY(dalloc(ctx, &ctx->node_off_d, n_inst + 1));
  TRY(dalloc(ctx, &ctx->ionic_d, 6 * n_inst));
  HIPC(hipMemcpyAsync(ctx->rowptr, ctx->host.rowptr.data(), (N + 1) * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->colidx, ctx->host.col.data(), nnz * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->diagpos, ctx->host.diag.data(), N * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->Aval, ctx->host.val.data(), nnz * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->ml, ctx->host.ml.data(), N * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->node_off_d, node_off, (n_inst + 1) * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->ionic_d, ionic, 6 * n_inst * 8, hipMemcpyHostToDevice, ctx->stream));
  if (emi) {
    TRY(dalloc(ctx, &ctx->emi_part, N));
    TRY(dalloc(ctx, &ctx->emi_sl, N));
    TRY(dalloc(ctx, &ctx->emi_ppos, N));
    TRY(dalloc(ctx, &ctx->emi_pmass, N));
    HIPC(hipMemcpyAsync(ctx->emi_part, emi_part.data(), N * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(ctx->emi_sl, emi_sl.data(), N * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(ctx->emi_ppos, emi_ppos.data(), N * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(ctx->emi_pmass, emi_pmass.data(), N * 8, hipMemcpyHostToDevice, ctx->stream));
    ctx->emi = true;
    ctx->emi_cm = emi->cm;
  }
  for (int m = 0; m < M; ++m)
    launch_build_h(ctx->stream, N, ctx->rowptr, ctx->diagpos, ctx->Aval, ctx->ml,
                   prm->dt * ctx->col.QI[m][m], ctx->Hval + m * nnz, ctx->dinv + m * N, ctx->emi_ppos,
                   ctx->emi_pmass);
  HIPC(hipGetLastError());
  TRY(build_dia(ctx));
  if (prm->format == 2 && ctx->nd == 0)
    return fail(ctx, SDC_ERR_ARG, "diagonal storage requested but a row pattern has more than %d offsets", kMaxDiag);
  if (prm->format == 3 && prm->scheme == 1)
    return fail(ctx, SDC_ERR_ARG, "the sliced ELL storage is not available with the linearized scheme");
  if ((prm->format == 0 || prm->format == 3) && prm->scheme == 0) TRY(build_sell(ctx));
  if (prm->format == 3 && !ctx->sell_ptr) return fail(ctx, SDC_ERR_ARG, "sliced ELL storage too large");

  const size_t MN = static_cast<size_t>(M) * N;
  TRY(dalloc(ctx, &ctx->v0, N));
  TRY(dalloc(ctx, &ctx->w0, N));
  for (double** b : {&ctx->v, &ctx->w, &ctx->I, &ctx->R, &ctx->Phi, &ctx->Gam, &ctx->dv, &ctx->dI, &ctx->dR})
    TRY(dalloc(ctx, b, MN));
  TRY(dalloc(ctx, &ctx->amax, N));
  TRY(dalloc(ctx, &ctx->p, N));
  for (int q = 0; q < 2; ++q) {
    TRY(dalloc(ctx, &ctx->r[q], N));
    TRY(dalloc(ctx, &ctx->wv[q], N));
    TRY(dalloc(ctx, &ctx->s[q], N));
  }

  // The XCD order of the work maps: chunks of about 8 stencil reaches (the
  // matrix bandwidth, in 256-row blocks), at least 4 blocks; a 3D grid's
  // reach of a plane makes the chunks an eighth of the map.
  {
    int64_t reach = 1;
    for (int64_t r = 0; r < N; ++r)
      for (int32_t e = ctx->host.rowptr[r]; e < ctx->host.rowptr[r + 1]; ++e)
        reach = std::max(reach, std::abs(static_cast<int64_t>(ctx->host.col[e]) - r));
    const int64_t chunk = std::max<int64_t>(4, (8 * reach + kBlock - 1) / kBlock);
    int sh = 0;
    while ((int64_t{1} << sh) < chunk && sh < kXcdContig) ++sh;
    ctx->xcd_shift = sh;
  }
  // all-rows work map (host-built)
  std::vector<BlkRec> rec;
  std::vector<int32_t> blk0(n_inst + 1), nblk(n_inst + 1), cnt(n_inst + 1), aoff(n_inst + 1);
  std::vector<int64_t> innz(n_inst + 1, 0);
  for (int i = 0; i < n_inst; ++i) {
    const int32_t lo = static_cast<int32_t>(node_off[i]), hi = static_cast<int32_t>(node_off[i + 1]);
    blk0[i] = static_cast<int32_t>(rec.size());
    cnt[i] = hi - lo;
    aoff[i] = lo;
    innz[i] = ctx->host.rowptr[hi] - ctx->host.rowptr[lo];
    nblk[i] = (hi - lo + kBlock - 1) / kBlock;
    for (int bi = 0; bi < nblk[i]; ++bi) {
      BlkRec r{};
      r.inst = i;
      r.beg = lo + bi * kBlock;
      r.end = std::min(r.beg + kBlock, hi);
      r.bi = bi;
      r.nb = nblk[i];
      r.lo = lo;
      r.hi = hi;
      for (int d = 0; d < ctx->nd; ++d) r.off[d] = ctx->dia_off_h[static_cast<size_t>(i) * ctx->nd + d];
      rec.push_back(r);
    }
  }
  aoff[n_inst] = static_cast<int32_t>(N);
  const int32_t nblk_all = static_cast<int32_t>(rec.size());
  TRY(alloc_map(ctx, &ctx->all, nblk_all));
  TRY(alloc_map(ctx, &ctx->dyn[0], nblk_all));
  TRY(alloc_map(ctx, &ctx->dyn[1], nblk_all));
  HIPC(hipMemcpyAsync(ctx->all.rec, rec.data(), rec.size() * sizeof(BlkRec), hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->all.inst_blk0, blk0.data(), n_inst * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->all.inst_nblk, nblk.data(), n_inst * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->all.inst_cnt, cnt.data(), n_inst * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->all.inst_nnz, innz.data(), n_inst * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->all.aoff, aoff.data(), (n_inst + 1) * 4, hipMemcpyHostToDevice, ctx->stream));
  ctx->all.nblk = nblk_all;
  ctx->all.rows = N;
  ctx->all.idx = nullptr;
  for (int i = 0; i < n_inst; ++i) {
    ctx->all.cnt[i] = cnt[i];
    ctx->all.nnz[i] = innz[i];
    ctx->all.max_nb = std::max(ctx->all.max_nb, nblk[i]);
  }
  TRY(dalloc(ctx, &ctx->list[0], static_cast<size_t>(nblk_all) * kBlock));
  TRY(dalloc(ctx, &ctx->list[1], static_cast<size_t>(nblk_all) * kBlock));
  for (int q = 0; q < 2; ++q) {
    TRY(dalloc(ctx, &ctx->cg_scal[q], static_cast<size_t>(kScal) * n_inst));
    if (q == 0) TRY(dalloc(ctx, &ctx->cg_tot, 4 * static_cast<size_t>(n_inst)));
    TRY(dalloc(ctx, &ctx->part[q], 4 * static_cast<size_t>(nblk_all)));
  }
  // done flags and iteration counts side by side: one copy reads both
  TRY(dalloc(ctx, &ctx->cg_done, 2 * static_cast<size_t>(n_inst)));
  ctx->cg_iters = ctx->cg_done + n_inst;
  TRY(dalloc(ctx, &ctx->wg_p, N));   // zero, and zero again after every workgroup solve
  if (prm->tol_sdc > 0.0) {
    TRY(dalloc(ctx, &ctx->e_part, static_cast<size_t>(M) * nblk_all));
    TRY(dalloc(ctx, &ctx->inst_energy, n_inst));
    TRY(dalloc(ctx, &ctx->inst_stop, n_inst));
    HIPC(hipHostMalloc(reinterpret_cast<void**>(&ctx->h_term), 2 * n_inst * sizeof(double)));
  }
  if (prm->scheme == 1) TRY(dalloc(ctx, &ctx->G, static_cast<size_t>(M) * N));
  if (prm->first_rings > 0) {
    TRY(dalloc(ctx, &ctx->carry_list, N));
    TRY(dalloc(ctx, &ctx->first_list, N));
    TRY(dalloc(ctx, &ctx->mark[0], N));
    TRY(dalloc(ctx, &ctx->mark[1], N));
  }
  if (prm->drop_mode == 1) {
    TRY(dalloc(ctx, &ctx->drop_part, 2 * static_cast<size_t>(nblk_all)));
    TRY(dalloc(ctx, &ctx->drop_theta, n_inst));
    TRY(dalloc(ctx, &ctx->drop_info, 4 * static_cast<size_t>(n_inst)));
  }
  TRY(dalloc(ctx, &ctx->cg_blk_done, nblk_all));
  TRY(dalloc(ctx, &ctx->sel_cnt, nblk_all));
  TRY(dalloc(ctx, &ctx->sel_nnz, nblk_all));
  HIPC(hipHostMalloc(reinterpret_cast<void**>(&ctx->h_i32), (8 + 2 * n_inst + 2 * M * n_inst) * sizeof(int32_t)));
  TRY(dalloc(ctx, &ctx->hist_done, 2 * static_cast<size_t>(M) * n_inst));
  ctx->hist_iters = ctx->hist_done + static_cast<size_t>(M) * n_inst;
  HIPC(hipHostMalloc(reinterpret_cast<void**>(&ctx->h_i64), map_sizes_words(n_inst) * sizeof(int64_t)));
  HIPC(hipStreamSynchronize(ctx->stream));
  // forward solves, reverse solves, forward solves of full-first-sweep steps
  // among heuristic ones
  ctx->pred.assign(3 * static_cast<size_t>(SDC_MAX_SWEEPS) * M, 8);
  ctx->coords_h.assign(coords, coords + N * dim);
  ctx->elems_h.assign(elems, elems + E * nv);
  ctx->tensor_h.assign(elem_tensor, elem_tensor + E * dim * dim);
  ctx->n_elem = E;
  TRY(autotune(ctx));
  TRY(tune_rows_per_thread(ctx));
  ctx->pin.assign(SDC_MAX_SWEEPS, nullptr);
  ctx->pin_n.assign(SDC_MAX_SWEEPS, 0);
  ctx->ready = true;
  return SDC_OK;
}

int sdc_add_stimulus(sdc_ctx* ctx, double t_on, const int32_t* nodes, int64_t n, double value) {
  TRY(check_ready(ctx));
  if (n < 0 || (n > 0 && !nodes)) return fail(ctx, SDC_ERR_ARG, "bad stimulus node list");
  for (int64_t q = 0; q < n; ++q)
    if (nodes[q] < 0 || nodes[q] >= ctx->N) return fail(ctx, SDC_ERR_ARG, "stimulus node out of range");
  Stimulus s{t_on, nullptr, n, value};
  HIPC(hipMalloc(reinterpret_cast<void**>(&s.nodes), std::max<int64_t>(n, 1) * sizeof(int32_t)));
  ctx->stims.push_back(s);
  HIPC(hipMemcpy(s.nodes, nodes, n * sizeof(int32_t), hipMemcpyHostToDevice));
  return SDC_OK;
}

int sdc_get_sizes(const sdc_ctx* ctx, int64_t* n, int64_t* nnz, int64_t* nw) {
  if (!ctx || !ctx->ready) return SDC_ERR_STATE;
  if (n) *n = ctx->N;
  if (nnz) *nnz = ctx->nnz;
  if (nw) *nw = ctx->N;
  return SDC_OK;
}

int sdc_get_system(sdc_ctx* ctx, int32_t* rowptr, int32_t* col, double* val, double* ml) {
  TRY(check_ready(ctx));
  if (rowptr) std::memcpy(rowptr, ctx->host.rowptr.data(), (ctx->N + 1) * 4);
  if (col) std::memcpy(col, ctx->host.col.data(), ctx->nnz * 4);
  if (val) std::memcpy(val, ctx->host.val.data(), ctx->nnz * 8);
  if (ml) std::memcpy(ml, ctx->host.ml.data(), ctx->N * 8);
  return SDC_OK;
}

int sdc_begin_step(sdc_ctx* ctx, const double* v, const double* w, double t) {
  TRY(check_ready(ctx));
  if (!v || !w) return fail(ctx, SDC_ERR_ARG, "null state");
  const int64_t N = ctx->N;
  // the rise record of the step before (if it continued its predecessor)
  ctx->rise_steps = (ctx->rise_steps << 1) | (ctx->rise_now ? 1u : 0u);
  ctx->rise_now = false;
  ctx->t_jump = !(ctx->t_known && std::fabs(t - ctx->t_next) <= 1e-6 * ctx->prm.dt);
  ctx->t_next = t + ctx->prm.dt;
  ctx->t_known = true;
  HIPC(hipMemcpyAsync(ctx->v0, v, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(ctx->w0, w, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  for (const auto& s : ctx->stims)
    if (stimulus_applies(s, t, ctx->prm.dt)) launch_set_values(ctx->stream, s.nodes, s.n, s.value, ctx->v0);
  TRY(build_first_set(ctx, t));
  return restart_step(ctx);
}

int sdc_sweep(sdc_ctx* ctx, sdc_sweep_stats* stats) {
  TRY(check_ready(ctx));
  if (!ctx->in_step) return fail(ctx, SDC_ERR_STATE, "sdc_sweep outside a step");
  if (ctx->k >= SDC_MAX_SWEEPS) return fail(ctx, SDC_ERR_STATE, "too many sweeps in one step");
  int rc = do_sweep(ctx, stats, true);
  if (rc != SDC_OK) ctx->in_step = false;
  return rc;
}

int sdc_end_step(sdc_ctx* ctx, double* v, double* w) {
  TRY(check_ready(ctx));
  if (!ctx->in_step) return fail(ctx, SDC_ERR_STATE, "sdc_end_step outside a step");
  if (!v || !w) return fail(ctx, SDC_ERR_ARG, "null state");
  const int64_t N = ctx->N, last = static_cast<int64_t>(ctx->prm.M - 1) * N;
  HIPC(hipMemcpyAsync(v, ctx->v + last, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(w, ctx->w + last, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->in_step = false;
  return SDC_OK;
}

int sdc_step(sdc_ctx* ctx, double* v, double* w, double t, sdc_step_stats* stats) {
  TRY(sdc_begin_step(ctx, v, w, t));
  // a step that does not continue the last one takes the synchronous loop
  // at once (its budget history belongs to another time)
  int first = ctx->t_jump ? 1 : 0;
  bool fresh = true;   // the step state is still as sdc_begin_step left it
  if (!ctx->t_jump && ctx->graph_usable()) {
    // graph-captured sweeps: one synchronisation per step; a short budget
    // redoes the step with the synchronous CG loop below
    bool short_budget = false;
    const int rc = graph_step(ctx, stats, &short_budget);
    if (rc != SDC_OK) {
      ctx->in_step = false;
      return rc;
    }
    if (!short_budget) return sdc_end_step(ctx, v, w);
    ++ctx->graph_redone;
    first = 1;
    fresh = false;
  }
  // fast path: predicted CG budgets, one synchronisation per sweep; if a
  // budget was short, redo the step from its saved start state with the
  // synchronous CG loop (identical results, exact iteration counts)
  for (int attempt = first; attempt < 2; ++attempt) {
    const bool async = attempt == 0;
    if (!fresh) {
      ++ctx->redone_steps;
      TRY(restart_step(ctx));
    }
    fresh = false;
    if (stats) std::memset(stats, 0, sizeof *stats);
    bool short_budget = false;
    for (int k = 0; k < ctx->prm.K; ++k) {
      int rc = do_sweep(ctx, stats ? &stats->sweep[k] : nullptr, k + 1 < ctx->prm.K, async, &short_budget);
      if (rc != SDC_OK) {
        ctx->in_step = false;
        return rc;
      }
      if (short_budget) break;
      if (stats) stats->n_sweeps = k + 1;
      if (ctx->terminate() && ctx->all_stopped) break;   // energy-norm termination
    }
    if (!short_budget) break;
  }
  return sdc_end_step(ctx, v, w);
}

int sdc_get_node(sdc_ctx* ctx, int32_t m, double* v_m, double* w_m) {
  TRY(check_ready(ctx));
  if (m < 0 || m >= ctx->prm.M) return fail(ctx, SDC_ERR_ARG, "node out of range");
  const int64_t N = ctx->N;
  if (v_m) HIPC(hipMemcpyAsync(v_m, ctx->v + m * N, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  if (w_m) HIPC(hipMemcpyAsync(w_m, ctx->w + m * N, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return SDC_OK;
}

int sdc_get_cg_iters(sdc_ctx* ctx, int32_t* out) {
  TRY(check_ready(ctx));
  if (!out) return fail(ctx, SDC_ERR_ARG, "null output");
  if (ctx->last_iters.empty()) return fail(ctx, SDC_ERR_STATE, "no sweep has run");
  std::memcpy(out, ctx->last_iters.data(), ctx->last_iters.size() * sizeof(int32_t));
  return SDC_OK;
}

int sdc_get_active(sdc_ctx* ctx, int32_t* idx, int64_t* n) {
  TRY(check_ready(ctx));
  const MapBuf& mb = ctx->curmap();
  if (n) *n = mb.rows;
  if (idx) {
    launch_map_rows(ctx->stream, mb.dev(), idx);
    HIPC(hipGetLastError());
  }
  return SDC_OK;
}

int sdc_set_active(sdc_ctx* ctx, int32_t sweep, const int32_t* idx, int64_t n) {
  TRY(check_ready(ctx));
  if (sweep < 0) {
    HIPC(hipStreamSynchronize(ctx->stream));
    for (auto& p : ctx->pin) {
      if (p) (void)hipFree(p);
      p = nullptr;
    }
    ctx->carry_n = -1;
    ctx->step_count = 0;
    return SDC_OK;
  }
  if (sweep == 0 || sweep >= SDC_MAX_SWEEPS || n < 0 || n > ctx->N || (n > 0 && !idx))
    return fail(ctx, SDC_ERR_ARG, "bad pinned set (sweep must be 1..%d)", SDC_MAX_SWEEPS - 1);
  if (!ctx->pin[sweep]) HIPC(hipMalloc(reinterpret_cast<void**>(&ctx->pin[sweep]), std::max<int64_t>(ctx->N, 1) * 4));
  if (n > 0) HIPC(hipMemcpyAsync(ctx->pin[sweep], idx, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->pin_n[sweep] = n;
  return SDC_OK;
}

int sdc_solve(sdc_ctx* ctx, int32_t m, const int32_t* idx, int64_t n, const double* b, double* x,
              int32_t* iters) {
  TRY(check_ready(ctx));
  if (m < 0 || m >= ctx->prm.M || n < 0 || n > ctx->N || !b || !x || (n > 0 && !idx))
    return fail(ctx, SDC_ERR_ARG, "bad solve arguments");
  ctx->in_step = false;   // the step's work vectors are reused
  const int64_t N = ctx->N;
  HIPC(hipMemsetAsync(x, 0, N * 8, ctx->stream));
  for (int q = 0; q < 2; ++q) {
    HIPC(hipMemsetAsync(ctx->r[q], 0, N * 8, ctx->stream));
    HIPC(hipMemsetAsync(ctx->wv[q], 0, N * 8, ctx->stream));
    HIPC(hipMemsetAsync(ctx->s[q], 0, N * 8, ctx->stream));
  }
  TRY(map_list(ctx, 0, idx, n));
  const MapBuf& mb = ctx->dyn[0];
  launch_copy_b(ctx->stream, mb.dev(), b, ctx->r[0], x);
  HIPC(hipGetLastError());
  std::vector<int> it;
  TRY(run_cg(ctx, m, mb, x, -1, &it));
  if (iters)
    for (int i = 0; i < ctx->n_inst; ++i) iters[i] = it[i];
  HIPC(hipStreamSynchronize(ctx->stream));
  return SDC_OK;
}

int sdc_select(sdc_ctx* ctx, const double* amax, const int32_t* idx_in, int64_t n_in, double theta,
               int32_t* idx_out, int64_t* n_out) {
  TRY(check_ready(ctx));
  if (!amax || !idx_out || !n_out || n_in < 0 || n_in > ctx->N || (n_in > 0 && !idx_in))
    return fail(ctx, SDC_ERR_ARG, "bad select arguments");
  ctx->in_step = false;
  TRY(map_list(ctx, 0, idx_in, n_in));
  MapBuf& nm = ctx->dyn[1];
  ZeroVecs none{{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr}, nullptr, 0, 0};
  launch_select(ctx->stream, ctx->dyn[0].dev(), ctx->n_inst, ctx->rowptr, amax, theta, nullptr, ctx->sel_cnt,
                ctx->sel_nnz, ctx->list[1], idx_out, ctx->next(nm), none, nullptr);
  HIPC(hipGetLastError());
  TRY(fetch_map(ctx, &nm));
  *n_out = nm.rows;
  return SDC_OK;
}

int sdc_get_drop_tolerance(sdc_ctx* ctx, double* out) {
  TRY(check_ready(ctx));
  if (!out) return fail(ctx, SDC_ERR_ARG, "null argument");
  if (!ctx->apriori_drop()) return fail(ctx, SDC_ERR_STATE, "the a-priori drop tolerance is not enabled");
  HIPC(hipMemcpyAsync(out, ctx->drop_info, 4 * ctx->n_inst * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  return SDC_OK;
}

int sdc_set_coefficients(sdc_ctx* ctx, const double* node_sigma, const double* ionic) {
  TRY(check_ready(ctx));
  if (ctx->emi) return fail(ctx, SDC_ERR_STATE, "sdc_set_coefficients is not available for the cell-by-cell model");
  ctx->in_step = false;
  if (ionic)
    HIPC(hipMemcpyAsync(ctx->ionic_d, ionic, 6 * ctx->n_inst * 8, hipMemcpyHostToDevice, ctx->stream));
  if (node_sigma) {
    HostSystem hs;
    std::string e = assemble_p1(ctx->dim, ctx->N, ctx->coords_h.data(), ctx->n_elem, ctx->elems_h.data(),
                                ctx->tensor_h.data(), node_sigma, &hs);
    if (!e.empty()) return fail(ctx, SDC_ERR_ARG, "assembly: %s", e.c_str());
    if (hs.col != ctx->host.col) return fail(ctx, SDC_ERR_STATE, "pattern changed");
    ctx->host.val.swap(hs.val);
    const int64_t N = ctx->N, nnz = ctx->nnz;
    const int M = ctx->prm.M;
    HIPC(hipMemcpyAsync(ctx->Aval, ctx->host.val.data(), nnz * 8, hipMemcpyHostToDevice, ctx->stream));
    for (int m = 0; m < M; ++m)
      launch_build_h(ctx->stream, N, ctx->rowptr, ctx->diagpos, ctx->Aval, ctx->ml,
                     ctx->prm.dt * ctx->col.QI[m][m], ctx->Hval + m * nnz, ctx->dinv + m * N, nullptr, nullptr);
    HIPC(hipGetLastError());
    if (ctx->nd > 0) TRY(build_dia(ctx));
    TRY(fill_sell(ctx));
  }
  HIPC(hipStreamSynchronize(ctx->stream));
  return SDC_OK;
}

int sdc_get_info(sdc_ctx* ctx, sdc_info* out) {
  TRY(check_ready(ctx));
  if (!out) return fail(ctx, SDC_ERR_ARG, "null output");
  out->format = ctx->fmt();
  out->n_diagonals = ctx->nd;
  out->t_csr_us = ctx->t_csr_us;
  out->t_dia_us = ctx->t_dia_us;
  out->redone_steps = ctx->redone_steps;
  out->rows_per_thread = ctx->use_dia && ctx->pair_all && compiled_diagonals(ctx->nd) ? 2 : 1;
  out->t_rows1_us = ctx->t_rows_us[0];
  out->t_rows2_us = ctx->t_rows_us[1];
  out->graph_steps = ctx->graph_steps;
  out->graph_captures = ctx->graph_captures;
  out->graph_redone = ctx->graph_redone;
  out->t_sell_us = ctx->t_sell_us;
  out->xcd_chunk = ctx->xcd_shift >= sdc::kXcdContig ? 0 : 1 << ctx->xcd_shift;
  return SDC_OK;
}

int sdc_set_graph(sdc_ctx* ctx, int32_t enable) {
  TRY(check_ready(ctx));
  if (!enable) {
    ctx->graph_mode = false;
    graph_release(ctx);
    return SDC_OK;
  }
  if (ctx->emi || ctx->linearized() || ctx->terminate() || ctx->apriori_drop() || ctx->first_subset() ||
      ctx->prm.cg_energy_tol > 0.0)
    return fail(ctx, SDC_ERR_ARG, "graph-captured sweeps support the default options of the monodomain model "
                "(scheme 0, fixed sweep count and drop tolerance, every first sweep on all rows, residual CG stop)");
  const int K = ctx->prm.K, M = ctx->prm.M, ni = ctx->n_inst;
  if (!ctx->cap_stream) HIPC(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  if (!ctx->ghist) {
    TRY(dalloc(ctx, &ctx->ghist, 2 * static_cast<size_t>(K) * M * ni));
    HIPC(hipHostMalloc(reinterpret_cast<void**>(&ctx->gh_hist), 2 * static_cast<size_t>(K) * M * ni * sizeof(int32_t)));
    HIPC(hipHostMalloc(reinterpret_cast<void**>(&ctx->gh_sizes), K * map_sizes_words(ni) * sizeof(int64_t)));
    ctx->gev.assign(K + 1, nullptr);
    for (auto& e : ctx->gev) HIPC(hipEventCreate(&e));
    HIPC(hipStreamSynchronize(ctx->stream));
  }
  ctx->graph_mode = true;
  ctx->graph_ready = false;
  return SDC_OK;
}

int sdc_profile(sdc_ctx* ctx, int32_t enable) {
  TRY(check_ready(ctx));
  if (enable && ctx->ev.empty()) {
    const int n = 2 * 4096;
    ctx->ev.resize(n);
    for (int i = 0; i < n; ++i) HIPC(hipEventCreate(&ctx->ev[i]));
  }
  ctx->prof = enable != 0;
  if (enable) ctx->pst = sdc_profile_stats{};
  return SDC_OK;
}

int sdc_profile_read(sdc_ctx* ctx, sdc_profile_stats* out) {
  TRY(check_ready(ctx));
  if (!out) return fail(ctx, SDC_ERR_ARG, "null output");
  *out = ctx->pst;
  return SDC_OK;
}

}  // extern "C"
