// Reverse (adjoint) SDC step: sdc_adjoint_step.
//
// Differentiates one step (v_n, w_n; sigma, a) -> (v_{n+1}, w_{n+1}) with the
// active sets of its sweeps held fixed, each restricted solve taken as exact.
// The step is first recomputed from (v_n, w_n) with the same kernels,
// recording every sweep's start values, corrections and active set (the
// forward is deterministic, so the sets are those of the original step);
// then the sweeps are reversed, last to first, node by node (last to first).
// H_m is symmetric, so the reverse solve is the same restricted Jacobi-PCG.
// Sensitivities: per-row accumulation for the Aliev-Panfilov parameter a
// (reduced per instance at the end) and per-element accumulation of
// psi^T Khat_T u for the nodal conductivity multipliers (gathered to the
// nodes at the end), so every sum has a fixed order.
#include <cstring>

#include "context.hpp"

using namespace sdc;

namespace {

int adjoint_setup(sdc_ctx* ctx) {
  if (ctx->emi) return fail(ctx, SDC_ERR_STATE, "the reverse pass is not available for the cell-by-cell model");
  if (ctx->terminate())
    return fail(ctx, SDC_ERR_STATE, "the reverse pass needs a fixed sweep count (no energy-norm termination)");
  if (ctx->linearized())
    return fail(ctx, SDC_ERR_STATE, "the reverse pass differentiates the implicit-explicit scheme (scheme 0)");
  if (ctx->first_subset())
    return fail(ctx, SDC_ERR_STATE, "the reverse pass needs first sweeps on all rows (first_rings = 0)");
  if (ctx->prm.cg_energy_tol > 0.0)
    return fail(ctx, SDC_ERR_STATE, "the reverse pass needs solves to the residual tolerance (cg_energy_tol = 0)");
  auto& A = ctx->adj;
  if (A.ready) return SDC_OK;
  const int nv = ctx->dim + 1, np = nv * ctx->dim / 2;
  const int64_t N = ctx->N, E = ctx->n_elem;
  const int M = ctx->prm.M, K = ctx->prm.K;
  std::vector<double> w;
  std::string e = element_pairs(ctx->dim, ctx->coords_h.data(), E, ctx->elems_h.data(), ctx->tensor_h.data(), &w);
  if (!e.empty()) return fail(ctx, SDC_ERR_ARG, "element data: %s", e.c_str());
  // node -> elements, ascending element order
  std::vector<int32_t> nptr(N + 1, 0), nel(static_cast<size_t>(E) * nv);
  for (int64_t q = 0; q < E * nv; ++q) nptr[ctx->elems_h[q] + 1]++;
  for (int64_t i = 0; i < N; ++i) nptr[i + 1] += nptr[i];
  {
    std::vector<int32_t> fill(nptr.begin(), nptr.end() - 1);
    for (int64_t el = 0; el < E; ++el)
      for (int a = 0; a < nv; ++a) nel[fill[ctx->elems_h[el * nv + a]]++] = static_cast<int32_t>(el);
  }
  TRY(dalloc(ctx, &A.elems, static_cast<size_t>(E) * nv));
  TRY(dalloc(ctx, &A.pairw, static_cast<size_t>(E) * np));
  TRY(dalloc(ctx, &A.nptr, N + 1));
  TRY(dalloc(ctx, &A.nel, static_cast<size_t>(E) * nv));
  HIPC(hipMemcpyAsync(A.elems, ctx->elems_h.data(), E * nv * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(A.pairw, w.data(), E * np * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(A.nptr, nptr.data(), (N + 1) * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(A.nel, nel.data(), E * nv * 4, hipMemcpyHostToDevice, ctx->stream));
  const size_t MN = static_cast<size_t>(M) * N;
  (void)K;
  for (double** b : {&A.Lv, &A.Lw, &A.Ldv, &A.Ldw}) TRY(dalloc(ctx, b, MN));
  for (double** b : {&A.Lv0, &A.Lw0, &A.psi, &A.u, &A.ga_row}) TRY(dalloc(ctx, b, N));
  TRY(dalloc(ctx, &A.qe, E));
  TRY(dalloc(ctx, &A.in_set, N));
  HIPC(hipStreamSynchronize(ctx->stream));   // host staging vectors go out of scope
  A.slots.resize(SDC_MAX_RECORDINGS);
  A.ready = true;
  return SDC_OK;
}

int ensure_slot(sdc_ctx* ctx, int slot) {
  if (slot < 0 || slot >= SDC_MAX_RECORDINGS) return fail(ctx, SDC_ERR_ARG, "recording slot out of range");
  auto& R = ctx->adj.slots[slot];
  if (R.v) return SDC_OK;
  const int M = ctx->prm.M, K = ctx->prm.K;
  const size_t MN = static_cast<size_t>(M) * ctx->N;
  TRY(dalloc(ctx, &R.v, (K + 1) * MN));
  TRY(dalloc(ctx, &R.w, (K + 1) * MN));
  TRY(dalloc(ctx, &R.dv, K * MN));
  TRY(dalloc(ctx, &R.list, static_cast<size_t>(K) * ctx->N));
  R.n.assign(K, -1);
  return SDC_OK;
}

// Recompute the step from (v, w) at time t, recording what the reverse needs
// into `slot`.  The end state stays in the context's last collocation node.
int record_step(sdc_ctx* ctx, int slot, const double* v, const double* w, double t) {
  TRY(ensure_slot(ctx, slot));
  auto& A = ctx->adj.slots[slot];
  A.valid = false;
  A.t = t;
  const int M = ctx->prm.M, K = ctx->prm.K;
  const int64_t N = ctx->N;
  const size_t MN = static_cast<size_t>(M) * N;
  TRY(sdc_begin_step(ctx, v, w, t));
  // predicted budgets when t continues the last step begun, else (the first
  // step of a segment recomputed from its checkpoint) the synchronous loop
  const int first = ctx->t_jump ? 1 : 0;
  for (int attempt = first; attempt < 2; ++attempt) {
    const bool async = attempt == 0;
    if (attempt > first) TRY(restart_step(ctx));
    bool short_budget = false;
    for (int k = 0; k < K && !short_budget; ++k) {
      const MapBuf& mb = ctx->curmap();
      if (mb.idx) {
        launch_map_rows(ctx->stream, mb.dev(), A.list + k * N);
        HIPC(hipGetLastError());
        A.n[k] = mb.rows;
      } else {
        A.n[k] = -1;
      }
      HIPC(hipMemcpyAsync(A.v + k * MN, ctx->v, MN * 8, hipMemcpyDeviceToDevice, ctx->stream));
      HIPC(hipMemcpyAsync(A.w + k * MN, ctx->w, MN * 8, hipMemcpyDeviceToDevice, ctx->stream));
      ctx->record_dv = A.dv + k * MN;
      int rc = do_sweep(ctx, nullptr, k + 1 < K, async, &short_budget);
      ctx->record_dv = nullptr;
      if (rc != SDC_OK) {
        ctx->in_step = false;
        return rc;
      }
    }
    if (!short_budget) break;
  }
  HIPC(hipMemcpyAsync(A.v + K * MN, ctx->v, MN * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(A.w + K * MN, ctx->w, MN * 8, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->in_step = false;
  A.valid = true;
  return SDC_OK;
}

// Reverse the step recorded in `slot`.
int reverse_step(sdc_ctx* ctx, int slot, double* lam_v, double* lam_w, double* g_sigma, double* g_a) {
  auto& A = ctx->adj;
  const auto& Rec = A.slots[slot];
  if (!Rec.valid) return fail(ctx, SDC_ERR_STATE, "recording slot %d holds no step", slot);
  const double t = Rec.t;
  const int M = ctx->prm.M, K = ctx->prm.K, nv = ctx->dim + 1;
  const int64_t N = ctx->N, E = ctx->n_elem;
  const size_t MN = static_cast<size_t>(M) * N;
  hipStream_t s = ctx->stream;

  // adjoints of the step's outputs: only the last node's values leave the step
  HIPC(hipMemsetAsync(A.Lv, 0, MN * 8, s));
  HIPC(hipMemsetAsync(A.Lw, 0, MN * 8, s));
  for (double* b : {A.Lv0, A.Lw0, A.psi, A.ga_row}) HIPC(hipMemsetAsync(b, 0, N * 8, s));
  HIPC(hipMemsetAsync(A.qe, 0, E * 8, s));
  HIPC(hipMemcpyAsync(A.Lv + (M - 1) * N, lam_v, N * 8, hipMemcpyDeviceToDevice, s));
  HIPC(hipMemcpyAsync(A.Lw + (M - 1) * N, lam_w, N * 8, hipMemcpyDeviceToDevice, s));

  const Map all = ctx->all.dev();
  const Mat Amat = ctx->A();
  std::vector<int> iters;
  const MapBuf* prev = nullptr;
  for (int k = K - 1; k >= 0; --k) {
    // CG work vectors must vanish off this sweep's set: clear the rows of the
    // set reversed last (the forward leaves them zero off the last set)
    if (prev) launch_zero_rows(s, prev->dev(), ctx->zv());
    const MapBuf* mb = &ctx->all;
    if (Rec.n[k] >= 0) {
      const int slot = (prev == &ctx->dyn[0]) ? 1 : 0;
      TRY(map_list(ctx, slot, Rec.list + k * N, Rec.n[k]));
      mb = &ctx->dyn[slot];
    }
    const Map map = mb->dev();
    HIPC(hipMemsetAsync(A.in_set, 0, N, s));
    launch_set_flags(s, map, A.in_set, 1);
    const double* V = Rec.v + k * MN;
    const double* W = Rec.w + k * MN;
    const double* Ve = Rec.v + (k + 1) * MN;
    const double* We = Rec.w + (k + 1) * MN;
    const double* DV = Rec.dv + k * MN;
    launch_adj_sweep_init(s, M, map, N, A.Lv, A.Lw, A.Ldv, A.Ldw);
    for (int m = M - 1; m >= 0; --m) {
      launch_adj_dw(s, M, m, map, N, ctx->ionic_d, V, W, Ve, We, A.Lv, A.Lw, A.Ldv, A.Ldw, A.Lw0, A.ga_row,
                    ctx->cargs);
      launch_copy_b(s, map, A.Ldv + m * N, ctx->r[0], A.psi);
      HIPC(hipGetLastError());
      const int slot = (SDC_MAX_SWEEPS + std::min(k, SDC_MAX_SWEEPS - 1)) * M + m;
      TRY(run_cg(ctx, m, *mb, A.psi, slot, &iters));
      launch_adj_apsi(s, M, m, all, N, Amat, ctx->ml, ctx->ionic_d, A.in_set, A.psi, V, W, Ve, We, DV, A.Lv, A.Lw,
                      A.Ldv, A.Ldw, A.Lv0, A.ga_row, A.u, ctx->cargs);
      launch_adj_elem(s, nv, E, A.elems, A.pairw, A.psi, A.u, A.qe);
      HIPC(hipGetLastError());
    }
    prev = mb;
  }
  launch_adj_spread(s, M, N, A.Lv, A.Lw, A.Lv0, A.Lw0);
  // a stimulus overwrite at the step start cuts the dependence on those values
  const double dt = ctx->prm.dt;
  for (const auto& st : ctx->stims)
    if (stimulus_applies(st, t, dt)) launch_zero_values(s, st.nodes, st.n, A.Lv0);
  HIPC(hipMemcpyAsync(lam_v, A.Lv0, N * 8, hipMemcpyDeviceToDevice, s));
  HIPC(hipMemcpyAsync(lam_w, A.Lw0, N * 8, hipMemcpyDeviceToDevice, s));
  launch_adj_gather_sigma(s, N, nv, A.nptr, A.nel, A.qe, g_sigma);
  launch_adj_reduce_a(s, ctx->n_inst, ctx->node_off_d, A.ga_row, g_a);
  HIPC(hipGetLastError());
  // the forward's work vectors hold reverse values now: the next step starts afresh
  if (prev) launch_zero_rows(s, prev->dev(), ctx->zv());
  return SDC_OK;
}

}  // namespace

extern "C" {

int sdc_adjoint_record(sdc_ctx* ctx, int32_t slot, double* v, double* w, double t) {
  TRY(check_ready(ctx));
  if (!v || !w) return fail(ctx, SDC_ERR_ARG, "null argument");
  TRY(adjoint_setup(ctx));
  TRY(record_step(ctx, slot, v, w, t));
  const int64_t N = ctx->N, last = static_cast<int64_t>(ctx->prm.M - 1) * N;
  HIPC(hipMemcpyAsync(v, ctx->v + last, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HIPC(hipMemcpyAsync(w, ctx->w + last, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return SDC_OK;
}

int sdc_adjoint_reverse(sdc_ctx* ctx, int32_t slot, double* lam_v, double* lam_w, double* g_sigma, double* g_a) {
  TRY(check_ready(ctx));
  if (!lam_v || !lam_w || !g_sigma || !g_a) return fail(ctx, SDC_ERR_ARG, "null argument");
  TRY(adjoint_setup(ctx));
  if (slot < 0 || slot >= SDC_MAX_RECORDINGS) return fail(ctx, SDC_ERR_ARG, "recording slot out of range");
  return reverse_step(ctx, slot, lam_v, lam_w, g_sigma, g_a);
}

int sdc_adjoint_step(sdc_ctx* ctx, const double* v_n, const double* w_n, double t, double* lam_v, double* lam_w,
                     double* g_sigma, double* g_a) {
  TRY(check_ready(ctx));
  if (!v_n || !w_n || !lam_v || !lam_w || !g_sigma || !g_a) return fail(ctx, SDC_ERR_ARG, "null argument");
  TRY(adjoint_setup(ctx));
  TRY(record_step(ctx, 0, v_n, w_n, t));
  return reverse_step(ctx, 0, lam_v, lam_w, g_sigma, g_a);
}

}  // extern "C"
