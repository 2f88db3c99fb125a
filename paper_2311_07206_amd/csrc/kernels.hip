// Device kernels of the adaptive SDC sweep (gfx950, wave64, FP64).
//
// Every active-row kernel is launched on a work map: block b owns up to
// kBlock consecutive positions of the active list of one instance, one row
// per thread.  Per-instance scalars (CG alpha/beta, norms) are reduced
// deterministically and without fences: each block writes one partial per
// quantity, and every block of the next launch sums its instance's partials
// in block order.  No floating-point atomics are used, so repeated runs are
// bitwise identical.
#include "kernels.hpp"
#include "device.hpp"

#include <hip/hip_ext.h>

#include <type_traits>

namespace sdc {

namespace {

// ------------------------------------------------------------------ helpers

// Butterfly over the wave, adjacent lanes first (the two-rows-per-thread CG
// kernel reproduces this order with the pair sum in the thread).
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum NV values over the block; the totals end up in thread 0's v[].
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* sh /* [4 * NV] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wid * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = (sh[k] + sh[NV + k]) + (sh[2 * NV + k] + sh[3 * NV + k]);
  }
}

// Visit the stored entries (value, column, is the row's diagonal) of row i
// of matrix A; f may ignore the third argument.  Storage S:
// 0 = CSR, -1 = diagonal storage with A.nd diagonals, S > 0 = diagonal
// storage with S diagonals known at compile time (fully unrolled, so all
// loads of the row are in flight together).  The diagonal offsets and the
// instance's row range come from the block's map entry.
constexpr int kCsrChunk = 8;

template <int S, class F>
__device__ __forceinline__ void for_entries(const Mat& A, int64_t N, const Row& rw, int i, F&& f) {
  if constexpr (S == 0) {
    // Entries in chunks of kCsrChunk whose loads are issued together: the
    // chunk's tail past the row's end reads the row's last entry with
    // weight 0 (adding exact zeros, so the sums equal the plain loop's).
    const int e0 = A.rowptr[i], e1 = A.rowptr[i + 1];
    for (int eb = e0; eb < e1; eb += kCsrChunk) {
      double a[kCsrChunk];
      int cq[kCsrChunk];
#pragma unroll
      for (int q = 0; q < kCsrChunk; ++q) {
        const int e = min(eb + q, e1 - 1);
        a[q] = A.val[e];
        cq[q] = A.col[e];
      }
#pragma unroll
      for (int q = 0; q < kCsrChunk; ++q) {
        const bool in = eb + q < e1;
        f(in ? a[q] : 0.0, cq[q], in && cq[q] == i);
      }
    }
  } else if constexpr (S == -2) {
    // Sliced ELL: the rows of a wavefront-sized slice hold their entries
    // column by column, so the 64 lanes of a wave on consecutive rows read
    // each entry position with one coalesced load.  Entries go in the row's
    // CSR order; past the row's length the slice's padding (value 0, the
    // row's own column) adds exact zeros, so the sums equal the CSR loop's.
    const int n_row = A.rowptr[i + 1] - A.rowptr[i];
    const int sl = i / kSlice, lane = i % kSlice;
    const int e0 = A.sptr[sl], len = (A.sptr[sl + 1] - e0) / kSlice;
    const double* vp = A.sval + e0 + lane;
    const int32_t* cp = A.scol + e0 + lane;
    for (int db = 0; db < len; db += kCsrChunk) {
      double a[kCsrChunk];
      int cq[kCsrChunk];
#pragma unroll
      for (int q = 0; q < kCsrChunk; ++q) {
        const int d = min(db + q, len - 1);
        a[q] = vp[d * kSlice];
        cq[q] = cp[d * kSlice];
      }
#pragma unroll
      for (int q = 0; q < kCsrChunk; ++q) {
        const bool in = db + q < len;
        f(in ? a[q] : 0.0, cq[q], in && db + q < n_row && cq[q] == i);
      }
    }
  } else {
    // Every load is unconditional (a column outside the instance reads row
    // i's own entry and is weighted 0), so that the compiler issues all of
    // them before the first wait.  Offset 0 sits at index h of the symmetric
    // offset list; its column is i itself.
    constexpr int kUnroll = S > 0 ? S : 1;
    const int nd = S > 0 ? S : A.nd;
    const int h = nd / 2;
#pragma unroll kUnroll
    for (int d = 0; d < nd; ++d) {
      const int c = d == h ? i : i + rw.off(d);
      const bool in = c >= rw.lo && c < rw.hi;
      const int k = in ? c : i;
      double a;
      if (d < h) {   // offset -o: the stored entry (c, c + o) of row c
        const double e = A.dval[(nd - 1 - d - h) * N + k];
        a = in ? e : 0.0;
      } else {
        a = A.dval[(d - h) * N + i];
      }
      f(a, k, d == h);
    }
  }
}

// Row i's stored entries under diagonal storage with S diagonals and its
// neighbours' values in the vectors u, w and (NS) s, read in a phase of its
// own: no arithmetic touches a loaded value before sums(), so a kernel that
// places a scheduling barrier between the two has every load in flight
// before its first wait.  sums() accumulates in for_entries<S>' order with
// its values (an entry whose column lies outside the instance counts 0), so
// the results agree bitwise.
template <int S, bool NS>
struct DiaLoads {
  static constexpr int h = S / 2;
  double a[S], gu[S], gw[S], gs[NS ? S : 1];
  bool in[S];
  __device__ __forceinline__ void load(const Mat& A, int64_t N, const Row& rw, int i, const double* __restrict__ u,
                                       const double* __restrict__ w, const double* __restrict__ s) {
#pragma unroll
    for (int d = 0; d < S; ++d) {
      const int c = d == h ? i : i + rw.off(d);
      in[d] = c >= rw.lo && c < rw.hi;
      const int k = in[d] ? c : i;
      a[d] = d < h ? A.dval[(S - 1 - d - h) * N + k] : A.dval[(d - h) * N + i];
      gu[d] = u[k];
      gw[d] = w[k];
      if constexpr (NS) gs[d] = s[k];
    }
  }
  __device__ __forceinline__ void sums(double& ar, double& aw, double& as, double& hii) const {
#pragma unroll
    for (int d = 0; d < S; ++d) {
      const double hv = d < h && !in[d] ? 0.0 : a[d];
      ar += hv * gu[d];
      aw += hv * gw[d];
      if constexpr (NS) as += hv * gs[d];
      if (d == h) hii = hv;
    }
  }
};

// Whether a CG kernel reading `rows` rows per thread under diagonal storage
// with S diagonals keeps its loads in one phase.  The kernels do so only with
// the instance totals formed beforehand (three loads instead of a thread's
// share of the partial sums, which would otherwise stay live across the phase)
// and while the loaded values fit the registers of a few waves per SIMD;
// beyond that the compiler's own interleaving of loads and arithmetic is the
// better schedule (measured on the 2D and 3D workloads).
template <int S, int rows>
constexpr bool phased_loads() { return S > 0 && 4 * S * rows <= 80; }

// Waves per SIMD the two-rows-per-thread kernel is compiled for: with more
// diagonals than a phase holds, a budget of two waves (256 registers) lets
// the compiler keep most of a row pair's loads in flight together instead of
// trading them for occupancy (the 19-diagonal 3D stencil runs faster so).
template <int S>
constexpr int pair_max_waves() { return phased_loads<S, 2>() ? 8 : 2; }

// Storage tags compiled: CSR (0), sliced ELL (-2), diagonal storage with 3
// (1D), 7 (2D triangles) or 19 (3D five-tet) diagonals, and diagonal storage
// with a runtime count (-1).
template <class F>
void dispatch_nd(int nd, F&& f) {
  switch (nd) {
    case 0: f(std::integral_constant<int, 0>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 19: f(std::integral_constant<int, 19>{}); break;
    default: f(std::integral_constant<int, -1>{}); break;
  }
}

template <class F>
void dispatch_storage(const Mat& A, F&& f) {
  if (A.nd == 0 && A.sptr)
    f(std::integral_constant<int, -2>{});
  else
    dispatch_nd(A.nd, f);
}

// Aliev-Panfilov current and gating rate (paper Sec. 5.1).
__device__ inline void ap_eval(double v, double w, const double* p, double& I, double& R) {
  const double k = p[0], a = p[1], eps0 = p[2], mu1 = p[3], mu2 = p[4], s = p[5];
  I = k * v * (v - a) * (v - 1.0) + v * w;
  R = s * (eps0 + mu1 * w / (v + mu2)) * (-w - k * v * (v - a - 1.0));
}

// dI/dv of the Aliev-Panfilov current: k ((v-a)(v-1) + v(v-1) + v(v-a)) + w.
__device__ inline double ap_didv(double v, double w, const double* p) {
  const double k = p[0], a = p[1];
  return k * ((v - a) * (v - 1.0) + v * (v - 1.0) + v * (v - a)) + w;
}

template <class F>
void dispatch_m(int M, F&& f) {
  switch (M) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    default: break;
  }
}

// ------------------------------------------------------------------ kernels

// Spread: every collocation value starts at the step's initial state.  With
// the cell-by-cell model the currents live on membrane sites (intracellular
// node, transmembrane voltage u_i - u_e); other nodes carry none.
template <int M, bool EMI>
__global__ __launch_bounds__(kBlock) void k_spread(Map map, int64_t N, const double* __restrict__ ionic,
                                                   const double* __restrict__ v0,
                                                   const double* __restrict__ w0, double* v,
                                                   double* w, double* I, double* R, EmiArgs e) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  const double a = v0[i], b = w0[i];
  double In = 0.0, Rn = 0.0;
  if constexpr (EMI) {
    if (e.sl[i] > 0.0) ap_eval(a - v0[e.part[i]], b, ionic + 6 * rw.inst, In, Rn);
  } else {
    ap_eval(a, b, ionic + 6 * rw.inst, In, Rn);
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    v[m * N + i] = a;
    w[m * N + i] = b;
    I[m * N + i] = In;
    R[m * N + i] = Rn;
  }
}

// Node that holds the membrane site of node i (cell-by-cell model).
__device__ inline int site_of(const EmiArgs& e, int i, double l) {
  return l > 0.0 ? i : (l < 0.0 ? e.part[i] : i);
}

__global__ void k_set_values(const int32_t* __restrict__ nodes, int64_t n, double value, double* v) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t < n) v[nodes[t]] = value;
}

// Sweep-start residuals on active rows (eq. final-sdc, right-hand sides):
//   F_j   = -(A v_j)_i - ML_i I_j,i
//   Phi_m = ML_i (v0_i - v_m,i) + dt sum_j Q[m][j] F_j
//   Gam_m = w0_i - w_m,i + dt sum_j Q[m][j] R_j,i
// and amax_i = 0 for this sweep's selection.
// Cell-by-cell model: ML I_j becomes sl I_j(site) and ML (v0 - v_m) the
// membrane mass cm |sl| ((v0 - v_m)_i - (v0 - v_m)_partner).
template <int M, int S, bool EMI>
__global__ __launch_bounds__(kBlock) void k_sweep_start(
    Map map, int64_t N, Mat A, const double* __restrict__ ml, const double* __restrict__ v0,
    const double* __restrict__ w0, const double* __restrict__ v, const double* __restrict__ w,
    const double* __restrict__ I, const double* __restrict__ R, double* __restrict__ Phi,
    double* __restrict__ Gam, double* __restrict__ amax, CollArgs c, EmiArgs e) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  double Av[M];
#pragma unroll
  for (int j = 0; j < M; ++j) Av[j] = 0.0;
  for_entries<S>(A, N, rw, i, [&](double a, int k, bool) {
#pragma unroll
    for (int j = 0; j < M; ++j) Av[j] += a * v[j * N + k];
  });
  const double mli = ml[i];
  double rwt = mli;   // weight of the site current in this row
  int site = i, pt = i;
  if constexpr (EMI) {
    const double l = e.sl[i];
    rwt = l;
    site = site_of(e, i, l);
    pt = l != 0.0 ? e.part[i] : i;
  }
  double F[M], Rj[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    F[j] = -Av[j] - rwt * I[j * N + site];
    Rj[j] = R[j * N + i];
  }
  const double v0i = v0[i], w0i = w0[i], v0p = v0[pt];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double sf = 0.0, sr = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      sf += c.Q[m][j] * F[j];
      sr += c.Q[m][j] * Rj[j];
    }
    double mass;
    if constexpr (EMI)
      mass = mli * ((v0i - v[m * N + i]) - (v0p - v[m * N + pt]));
    else
      mass = mli * (v0i - v[m * N + i]);
    Phi[m * N + i] = mass + c.dt * sf;
    Gam[m * N + i] = w0i - w[m * N + i] + c.dt * sr;
  }
  amax[i] = 0.0;
}

// Right-hand side of node m; CG start values x = 0, r = b on active rows:
//   b_i = Phi_m,i - dt ML_i sum_{j<m} QE[m][j] dI_j,i - dt sum_k A_ik sum_{j<m} QI[m][j] dv_j,k
// or, in the linearized scheme (LIN, G = ML dI/dv at the sweep's iterate),
//   b_i = Phi_m,i - dt sum_{j<m} QI[m][j] G_j,i dv_j,i - dt sum_k A_ik sum_{j<m} QI[m][j] dv_j,k.
template <int M, int S, bool EMI, bool LIN>
__global__ __launch_bounds__(kBlock) void k_rhs(Map map, int m, int64_t N, Mat A,
                                                const double* __restrict__ ml,
                                                const double* __restrict__ Phi_m,
                                                const double* __restrict__ dI,
                                                const double* __restrict__ dv, double* __restrict__ r,
                                                double* __restrict__ x, CollArgs c, EmiArgs e,
                                                const double* __restrict__ G) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  double ay = 0.0;
  if (m > 0) {
    for_entries<S>(A, N, rw, i, [&](double a, int k, bool) {
      double y = 0.0;
#pragma unroll
      for (int j = 0; j < M - 1; ++j)
        if (j < m) y += c.QI[m][j] * dv[j * N + k];
      ay += a * y;
    });
  }
  double rwt;
  int site = i;
  if constexpr (EMI) {
    rwt = e.sl[i];
    site = site_of(e, i, rwt);
  } else {
    rwt = ml[i];
  }
  double ex = 0.0;
  if constexpr (LIN) {
#pragma unroll
    for (int j = 0; j < M - 1; ++j)
      if (j < m) ex += c.QI[m][j] * (G[j * N + i] * dv[j * N + i]);
    r[i] = Phi_m[i] - c.dt * ex - c.dt * ay;
  } else {
#pragma unroll
    for (int j = 0; j < M - 1; ++j)
      if (j < m) ex += c.QE[m][j] * dI[j * N + site];
    r[i] = Phi_m[i] - c.dt * rwt * ex - c.dt * ay;
  }
  x[i] = 0.0;
}

// CG start from a given right-hand side b (component solve): r = b, x = 0.
__global__ __launch_bounds__(kBlock) void k_copy_b(Map map, const double* __restrict__ bvec,
                                                   double* __restrict__ r, double* __restrict__ x) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  r[rw.row] = bvec[rw.row];
  x[rw.row] = 0.0;
}

// Jacobi-PCG in the single-reduction (Chronopoulos-Gear) arrangement: with
// u = dinv r, w = H u and s = H p carried along, one iteration is
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u = dinv r,  w = H u,  gamma = r.u,  delta = w.u,  rr = r.r,
// with beta = gamma / gamma_old and alpha = gamma / (delta - beta gamma / alpha_old):
// the iterates of standard PCG in exact arithmetic, with one global
// reduction per iteration.  The vectors are kept scaled by the
// preconditioner, u = dinv r, w~ = dinv w, s~ = dinv s (double-buffered;
// zero on inactive rows, which is the restricted solve's Dirichlet
// condition), so the new H u = H dinv r - alpha H dinv (w + beta s) is a
// sum over the row's entries of h times u, w~ and s~ of the column: four
// loads per entry, no gather of dinv.  The row's own residual is
// r = H_ii u.
//
// Reductions without fences: every block writes its partial sums; each block
// of the next launch sums the partials of its instance in block order (so
// every block obtains bitwise the same scalars) and block 0 of the instance
// records the scalars, the stopping decision and the iteration count.
// Launch `it` first tests the residual left by `it` updates, then performs
// update it+1; a solve that stops after n updates therefore takes n + 1
// launches.

struct CgBufs {
  double* part[2];     // [nblk][4] partial sums written by launch parity
  double* scal[2];     // [n_inst][kScal] scalars written by launch parity
};

template <int NV>
__device__ inline void write_partials(double (&v)[NV], int blk, double* part, double* sh) {
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) part[4 * blk + q] = v[q];
  }
}

// Start from r0 = b: u0 = dinv r0 and w~0 = dinv H u0 (written for the first
// iteration); partials of gamma0 = r0.u0, delta0 = w0.u0, bb = r0.r0.
template <int S>
__global__ __launch_bounds__(kBlock) void k_cg_start(Map map, int n_inst, int64_t N, Mat H,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ r0,
                                                     double* __restrict__ u0, double* __restrict__ w0,
                                                     double* part_out, CgState cg) {
  __shared__ double sh[16];
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < n_inst; t += kBlock) {
      cg.done[t] = map.inst_nblk[t] == 0 ? 1 : 0;   // no active rows: nothing to solve
      cg.iters[t] = 0;
    }
  }
  if (static_cast<int>(blockIdx.x) >= map.nblk) return;
  const Row rw = map_row(map);
  if (rw.dead) return;
  if (threadIdx.x == 0) cg.blk_done[rw.blk] = 0;
  double s[3] = {0.0, 0.0, 0.0};
  if (rw.valid) {
    const int i = rw.row;
    double acc = 0.0;
    for_entries<S>(H, N, rw, i, [&](double h, int k, bool) { acc += h * (dinv[k] * r0[k]); });
    const double di = dinv[i], ri = r0[i], ui = di * ri;
    u0[i] = ui;
    w0[i] = di * acc;
    s[0] = ri * ui;
    s[1] = acc * ui;
    s[2] = ri * ri;
  }
  write_partials<3>(s, rw.blk, part_out, sh);
}

// Block total of NV values, formed by every thread in the same order
// (bitwise the total block_sum leaves in thread 0).  One barrier.
template <int NV>
__device__ inline void block_total(double (&v)[NV], double* sh /* [4 * NV] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wid * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = (sh[k] + sh[NV + k]) + (sh[2 * NV + k] + sh[3 * NV + k]);
}

// One launch per iteration; FIRST is launch 0 (beta = 0, no previous p, s).
// XW: launches of odd index read and write the iterate x, applying their own
// update and the one the launch before deferred (x_k = x_{k-1} + alpha_k p_k
// from the previous launch's alpha and p, then this launch's update, in that
// order, so x is bitwise that of one update per launch); launches of even
// index leave x, and a launch that finds the stop writes the deferred update.
// The direction p is deferred likewise: launches of even index neither read
// nor write it, and the next launch forms their p again, bitwise, from the
// same operands.
// Memory round trips before the arithmetic: (1) the block record, the list
// entry of the thread's row and the block's stop flag; (2) everything else
// the iteration reads: the instance's partial sums and scalars from the
// previous launch and the row's values and neighbour sums over the scaled vectors
//   a_r = sum_k h_ik u_k,  a_w = sum_k h_ik w~_k,  a_s = sum_k h_ik s~_k,
// so that H u of the new residual, u = dinv (r - alpha (w + beta s)), is
// a_r - alpha (a_w + beta a_s).
// Threads past the block's last row load row 0's values (in bounds) and
// contribute zeros.
// The arguments the first round trip needs come first, as plain pointers and
// integers, so that they can be preloaded into scalar registers at wave
// launch (the library is built with kernel-argument preloading).
// Per-instance totals of a launch's partial sums (one block per instance),
// in the order the iteration kernel would sum them.
__global__ __launch_bounds__(kBlock) void k_cg_totals(const int32_t* __restrict__ inst_blk0,
                                                      const int32_t* __restrict__ inst_nblk,
                                                      const double* __restrict__ part, double* __restrict__ tot) {
  __shared__ double sh[16];
  const int inst = blockIdx.x, b0 = inst_blk0[inst], nb = inst_nblk[inst];
  double acc[3] = {0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 3 * kBlock < nb; b += 4 * kBlock) {   // four independent loads in flight
    double v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 3; ++k) v[q][k] = part[4 * (b0 + b + q * kBlock) + k];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] += v[q][k];
  }
  for (; b < nb; b += kBlock)
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] += part[4 * (b0 + b) + k];
  block_total<3>(acc, sh);
  if (threadIdx.x < 3) tot[4 * inst + threadIdx.x] = acc[threadIdx.x];
}

// Energy-error stop of launch `it` >= 1 (stop.delay >= 1): the step terms
// t_j = alpha_j gamma_j for j < it are t_{it-1} from the previous launch's
// scalars (sc) and the earlier ones from its ring.  Returns the running sum
// sum_{j<it} t_j in e_sum and t_{it-1} in e_last, and whether the last
// min(d, it) terms, summed left to right, are at most etol2 times it (the
// test applies from it >= d).
__device__ inline bool energy_stop(const double* sc, double sc_alpha, double sc_rz, int it, const CgStop& stop,
                                   double& e_sum, double& e_last) {
  const int d = stop.delay;
  e_last = sc_alpha * sc_rz;
  e_sum = sc[kE] + e_last;
  double win = 0.0;
  for (int j = max(it - d, 0); j < it - 1; ++j) win += sc[kRing + j % d];
  win += e_last;
  return it >= d && win <= stop.etol2 * e_sum;
}

// Block 0 of the instance carries the running sum and the ring forward.
__device__ inline void energy_record(const double* sc, double* so, bool first, int it, int d, double e_sum,
                                     double e_last) {
  if (first) {
    so[kE] = 0.0;
    return;
  }
  so[kE] = e_sum;
  for (int q = 0; q < d; ++q) so[kRing + q] = sc[kRing + q];
  so[kRing + (it - 1) % d] = e_last;
}

// TOT: 0 the kernel sums its instance's partial sums (loads issued with the
// row's values); 1 it reads the instance's totals (k_cg_totals ran first);
// 2 it sums the partial sums itself once its stencil sums are formed, in
// the order of k_cg_totals (bitwise the same totals, without that launch),
// and reads the values only the update needs after that.
template <int S, bool FIRST, int LIST, int TOT, bool XW>
__global__ __launch_bounds__(kBlock) void k_cg_iter(int32_t* __restrict__ blk_done, const BlkRec* __restrict__ rec,
                                                    const int32_t* __restrict__ idx, int nblk, int xcd_shift,
                                                    const int32_t* __restrict__ live, int it,
                                                    const double* __restrict__ part_in,
                                                    const double* __restrict__ scal_in, int64_t N, Mat H,
                                                    const double* __restrict__ dinv,
                                                    double* __restrict__ x, double* __restrict__ p,
                                                    const double* __restrict__ u_in,
                                                    const double* __restrict__ w_in,
                                                    const double* __restrict__ s_in,
                                                    double* __restrict__ u_out,
                                                    double* __restrict__ w_out,
                                                    double* __restrict__ s_out,
                                                    double* __restrict__ part_out,
                                                    double* __restrict__ scal_out, CgStop stop,
                                                    int32_t* __restrict__ done, int32_t* __restrict__ iters) {
  __shared__ double sh_in[16], sh_out[16];
  // first round trip: the block's map entry and stop flag, the list entry of the thread's row
  const Map map{rec, nullptr, nullptr, idx, nblk, 0, live, xcd_shift};
  const Row rw = map_row<LIST>(map);
  const int L = rw.blk;
  // Early exit of a stopped block (or one past a live map's entries).  The
  // test includes invariants of the arguments (it >= 0, nd >= 0, output
  // buffers given) and of the list (entries >= 0), so that every cache line
  // of the kernel arguments and the list entry are read before the branch
  // rather than after it.
  if (rw.dead | blk_done[L] | (it < 0) | (H.nd < 0) | (rw.listed < 0) | (s_out == nullptr) | (iters == nullptr))
    return;
  const int inst = rw.inst, nb = rw.nb, b0 = L - rw.bi;
  const bool valid = rw.valid;
  const int i = rw.row;
  // second round trip, issued together: the row's values and neighbour sums,
  // the instance's scalars and partial sums from the previous launch
  constexpr bool kPhased = TOT != 0 && phased_loads<S, 1>();
  double a_r = 0.0, a_w = 0.0, a_s = 0.0, hii = 0.0;
  DiaLoads<kPhased ? S : 1, !FIRST> dl;
  if constexpr (kPhased) {
    dl.load(H, N, rw, i, u_in, w_in, s_in);
  } else {
    for_entries<S>(H, N, rw, i, [&](double h, int k, bool diag) {
      a_r += h * u_in[k];
      a_w += h * w_in[k];
      if (!FIRST) a_s += h * s_in[k];
      if (diag) hii = h;
    });
  }
  const double si = FIRST ? 0.0 : s_in[i];
  const double ui = u_in[i], wi = w_in[i];
  // The direction p is kept, like x, by the launches of odd index only (a
  // row's p then costs 24 bytes per two launches instead of 32): such a
  // launch rebuilds the previous launch's p_{L-1} = u_{L-1} + beta_{L-1}
  // p_{L-2} from p_{L-2} (zero before the first launch), u_{L-1} (still in
  // this launch's output buffer) and beta_{L-1}, as that launch formed it.
  double p_prev2 = 0.0, u_prev = 0.0, x_old = 0.0;
  if constexpr (XW && TOT != 2) {
    p_prev2 = it > 1 ? p[i] : 0.0;
    u_prev = u_out[i];
    x_old = x[i];
  }
  double sc_rz = 0.0, sc_alpha = 0.0, sc_bb = 0.0, sc_beta = 0.0;
  const double* sc = scal_in + inst * kScal;
  if (!FIRST) {
    sc_rz = sc[kRZ];
    sc_alpha = sc[kAlpha];
    sc_bb = sc[kBB];
    sc_beta = sc[kBeta];
  }
  double acc[3] = {0.0, 0.0, 0.0};
  // The instance's totals (k_cg_totals) or, without them, its partial sums
  // (at most kTotBlocks): the first kq kBlock by unconditional loads at a
  // clamped index issued with the rest (weights in the arithmetic), further
  // ones in a loop of uniform trip count for instances of more blocks.
  // Terms of weight 0 add nothing, so skipping them leaves the sums bitwise
  // those of the full unrolled read.  Two rounds cover the listed sets of a
  // 2D batch (fewer registers); the 19-diagonal 3D sets span up to four and
  // keep them unrolled (measured faster).
  constexpr int kq = TOT != 0 ? 1 : S > 7 ? kTotBlocks / kBlock : 2;
  double pv[kq][3];
  if constexpr (TOT == 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) pv[0][k] = part_in[4 * inst + k];
  } else if constexpr (TOT == 0) {
#pragma unroll
    for (int q = 0; q < kq; ++q) {
      const int b = static_cast<int>(threadIdx.x) + q * kBlock;
      const double* pp = part_in + 4 * (b0 + min(b, nb - 1));
#pragma unroll
      for (int k = 0; k < 3; ++k) pv[q][k] = pp[k];
    }
  }
  if constexpr (kPhased) {
    __builtin_amdgcn_sched_barrier(0);   // every load above is issued before the arithmetic below
    dl.sums(a_r, a_w, a_s, hii);
    // the stencil sums formed here, before the partial sums are read (so
    // the row's loaded values are not kept alive across that read)
    if constexpr (TOT == 2) asm volatile("" : "+v"(a_r), "+v"(a_w), "+v"(a_s), "+v"(hii));
  }
  // the Jacobi factor from the row's diagonal, as the stored dinv was formed
  const double di = 1.0 / hii;
  if constexpr (TOT == 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] = pv[0][k];
  } else if constexpr (TOT == 2) {
    // the instance's partial sums (at most kTotBlocks), then the update's values
    __builtin_amdgcn_sched_barrier(0);
    for (int b = static_cast<int>(threadIdx.x); b < nb; b += kBlock)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] += part_in[4 * (b0 + b) + k];
    block_total<3>(acc, sh_in);
    if constexpr (XW) {
      p_prev2 = it > 1 ? p[i] : 0.0;
      u_prev = u_out[i];
      x_old = x[i];
    }
  } else {
#pragma unroll
    for (int q = 0; q < kq; ++q) {
      const int b = static_cast<int>(threadIdx.x) + q * kBlock;
      const double wgt = b < nb ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] += wgt * pv[q][k];
    }
    for (int q = kq; q * kBlock < nb; ++q) {   // nb <= kTotBlocks without totals
      const int b = static_cast<int>(threadIdx.x) + q * kBlock;
      const double* pp = part_in + 4 * (b0 + min(b, nb - 1));
      const double wgt = b < nb ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] += wgt * pp[k];
    }
    block_total<3>(acc, sh_in);
  }
  const double p_old = XW ? fma(sc_beta, p_prev2, u_prev) : 0.0;   // p_{L-1}
  const double gamma = acc[0], delta = acc[1], rr = acc[2];
  double alpha, beta, bb;
  if (FIRST) {
    bb = rr;
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    bb = sc_bb;
    beta = gamma / sc_rz;
    alpha = gamma / (delta - beta * gamma / sc_alpha);
  }
  double e_sum = 0.0, e_last = 0.0;
  const bool e_stop = !FIRST && stop.delay > 0 && energy_stop(sc, sc_alpha, sc_rz, it, stop, e_sum, e_last);
  int status = 0;
  if (!isfinite(rr)) status = 3;
  else if (rr <= stop.rtol2 * bb) status = 1;
  else if (e_stop) status = 1;
  else if (it >= stop.maxit) status = 2;
  else if (!isfinite(alpha) || !(alpha > 0.0)) status = 3;
  if (rw.bi == 0 && threadIdx.x == 0) {
    // block 0 of the instance records the outcome and the scalars
    done[inst] = status;
    iters[inst] = it;
    double* so = scal_out + inst * kScal;
    so[kRZ] = gamma;
    so[kAlpha] = alpha;
    so[kBB] = bb;
    so[kBeta] = beta;
    if (stop.delay > 0) energy_record(sc, so, FIRST, it, stop.delay, e_sum, e_last);
  }
  if (status != 0) {
    // the stop leaves x final: a launch of odd index applies the update the
    // launch before it deferred
    if (XW && valid) x[i] = fma(sc_alpha, p_old, x_old);
    if (threadIdx.x == 0) blk_done[L] = status;
    return;
  }
  double s[3] = {0.0, 0.0, 0.0};
  if (valid) {
    const double w_new = a_r - alpha * (a_w + beta * a_s);   // H u of the new residual
    const double sv = wi + beta * si;                         // dinv (w + beta s)
    if constexpr (XW) {
      const double pi = fma(beta, p_old, ui);
      x[i] = fma(alpha, pi, fma(sc_alpha, p_old, x_old));   // the deferred update, then this one
      p[i] = pi;
    }
    s_out[i] = sv;
    const double un = ui - alpha * sv;                        // dinv (r - alpha s)
    u_out[i] = un;
    w_out[i] = di * w_new;
    const double rn = hii * un;
    s[0] = rn * un;
    s[1] = w_new * un;
    s[2] = rn * rn;
  }
  write_partials<3>(s, L, part_out, sh_out);
}

// ---- the CG iteration on all rows of an instance, two adjacent rows per thread

constexpr int kPairThreads = kBlock / 2;

// Sum over a 128-thread block of per-thread values that are already the sum
// of the thread's two rows, in the order block_sum / block_total take over
// the same 256 rows at one row per lane (the adjacent-lane step is the pair
// sum, the remaining steps are the lane butterfly within 32 lanes, then the
// four 64-row groups), so both kernels produce bitwise the same block sums.
// The total ends in every thread.
template <int NV>
__device__ inline void pair_block_total(double (&v)[NV], double* sh /* [4 * NV] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) v[k] += __shfl_xor(v[k], off, 64);
  }
  if ((lane & 31) == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[(2 * wid + (lane >> 5)) * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = (sh[k] + sh[NV + k]) + (sh[2 * NV + k] + sh[3 * NV + k]);
}

// Stores of the outputs of a launch over every row.  Such a launch streams
// more data than the caches keep between launches (a batch's all-rows
// launch moves about 300 MB), so its outputs are written non-temporally and
// leave the L2 to the neighbour rows the stencil gathers still read; all-rows
// launches measured 7-12 % faster so.  Listed sets keep ordinary stores:
// their next launch reads the outputs back while the Infinity Cache still
// holds them (non-temporal stores made batched listed launches about 20 %
// slower).
__device__ inline void stream_store(double* a, double v) { __builtin_nontemporal_store(v, a); }

// k_cg_iter for maps without a list (every row of the instances: the first
// sweep of a step) and diagonal storage, with 128 threads per 256-row map
// entry.  Thread t owns rows beg + 2t and beg + 2t + 1; in blocks whose
// stencil stays inside the instance, every value of the two rows sits at
// adjacent addresses, so each pair is one 16-byte load and the address work
// per row halves.  Other blocks take the rows one after the other.  The
// arithmetic per row and the order of every sum are those of k_cg_iter, so
// the two kernels agree bitwise.
template <int S, bool FIRST, bool TOT, bool XW>
__global__ __launch_bounds__(kPairThreads) __attribute__((amdgpu_waves_per_eu(1, pair_max_waves<S>())))
void k_cg_iter2(int32_t* __restrict__ blk_done,
                const BlkRec* __restrict__ rec,
                const int32_t* __restrict__ idx, int nblk, int xcd_shift,
                const int32_t* __restrict__ live, int it,
                const double* __restrict__ part_in,
                const double* __restrict__ scal_in, int64_t N, Mat H,
                const double* __restrict__ dinv,
                double* __restrict__ x, double* __restrict__ p,
                const double* __restrict__ u_in,
                const double* __restrict__ w_in,
                const double* __restrict__ s_in,
                double* __restrict__ u_out,
                double* __restrict__ w_out,
                double* __restrict__ s_out,
                double* __restrict__ part_out,
                double* __restrict__ scal_out, CgStop stop,
                int32_t* __restrict__ done, int32_t* __restrict__ iters) {
  static_assert(S > 0, "diagonal storage with a compile-time count");
  __shared__ double sh_in[16], sh_out[16];
  const int L = logical_block(nblk, xcd_shift);
  const int t = static_cast<int>(threadIdx.x);
  Row rw;
  rw.word = reinterpret_cast<const int32_t*>(rec + L)[min(t & 63, kRecWords - 1)];
  rw.inst = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, inst) / 4);
  rw.beg = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, beg) / 4);
  rw.end = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, end) / 4);
  rw.bi = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, bi) / 4);
  rw.nb = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, nb) / 4);
  rw.lo = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, lo) / 4);
  rw.hi = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, hi) / 4);
  rw.blk = L;
  rw.listed = 0;
  if (blk_done[L] | (it < 0) | (H.nd < 0) | (s_out == nullptr) | (iters == nullptr) | (idx != nullptr)) return;
  const int inst = rw.inst, nb = rw.nb, b0 = L - rw.bi;
  const int n_rows = rw.end - rw.beg;
  const bool va = 2 * t < n_rows, vb = 2 * t + 1 < n_rows;
  const int ia = va ? rw.beg + 2 * t : 0, ib = vb ? rw.beg + 2 * t + 1 : 0;
  constexpr int h = S / 2;
  const bool interior = n_rows == kBlock && rw.beg + rw.off(0) >= rw.lo && rw.end - 1 + rw.off(S - 1) < rw.hi;
  double ar[2] = {0.0, 0.0}, aw[2] = {0.0, 0.0}, as[2] = {0.0, 0.0}, hii[2] = {0.0, 0.0};
  // x and p are kept by the launches of odd index only (see k_cg_iter); with
  // 19 diagonals this variant needs more registers than two waves per SIMD
  // allow and runs at one, measured faster than keeping p in every launch
  const bool p_read = XW && it > 1;
  double si[2], pld[2], uprev[2], pold[2], di[2], ui[2], wi[2], xold[2];
  double sc_rz = 0.0, sc_alpha = 0.0, sc_bb = 0.0, sc_beta = 0.0;
  const double* sc = scal_in + inst * kScal;
  double acc[3] = {0.0, 0.0, 0.0};
  if constexpr (TOT && phased_loads<S, 2>()) {
    // Everything the iteration reads is requested before the first wait: the
    // two rows' own values, the instance's scalars and totals (ahead of the
    // interior/edge branch, so that no load waits behind it), then the
    // stencil's values and neighbour sums.
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = q ? ib : ia;
      si[q] = FIRST ? 0.0 : s_in[i];
      ui[q] = u_in[i];
      wi[q] = w_in[i];
    }
    if (!FIRST) {
      sc_rz = sc[kRZ];
      sc_alpha = sc[kAlpha];
      sc_bb = sc[kBB];
      sc_beta = sc[kBeta];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] = part_in[4 * inst + k];
    if (interior) {
      // both rows valid, ib = ia + 1, every column inside the instance: each
      // pair of values is one 16-byte load; the offset-0 term takes the rows'
      // own values read above
      double hv[S][2], gu[S][2], gw[S][2], gs[FIRST ? 1 : S][2];
#pragma unroll
      for (int d = 0; d < S; ++d) {
        const double* hp = d < h ? H.dval + static_cast<int64_t>(S - 1 - d - h) * N + ia + rw.off(d)
                                 : H.dval + static_cast<int64_t>(d - h) * N + ia;
        hv[d][0] = hp[0];
        hv[d][1] = hp[1];
        if (d != h) {
          const int c = ia + rw.off(d);
          gu[d][0] = u_in[c];
          gu[d][1] = u_in[c + 1];
          gw[d][0] = w_in[c];
          gw[d][1] = w_in[c + 1];
          if constexpr (!FIRST) {
            gs[d][0] = s_in[c];
            gs[d][1] = s_in[c + 1];
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);   // every load above is issued before the arithmetic below
#pragma unroll
      for (int d = 0; d < S; ++d) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double hq = hv[d][q];
          ar[q] += hq * (d == h ? ui[q] : gu[d][q]);
          aw[q] += hq * (d == h ? wi[q] : gw[d][q]);
          if constexpr (!FIRST) as[q] += hq * (d == h ? si[q] : gs[d][q]);
          if (d == h) hii[q] = hq;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int i = q ? ib : ia;
        for_entries<S>(H, N, rw, i, [&](double hv, int k, bool diag) {
          ar[q] += hv * u_in[k];
          aw[q] += hv * w_in[k];
          if (!FIRST) as[q] += hv * s_in[k];
          if (diag) hii[q] = hv;
        });
      }
    }
  } else {
    if (interior) {
      // both rows valid, ib = ia + 1, every column inside the instance
#pragma unroll
      for (int d = 0; d < S; ++d) {
        const int c = ia + rw.off(d);
        const double* hp = d < h ? H.dval + static_cast<int64_t>(S - 1 - d - h) * N + c
                                 : H.dval + static_cast<int64_t>(d - h) * N + ia;
        const double h0 = hp[0], h1 = hp[1];
        ar[0] += h0 * u_in[c];
        ar[1] += h1 * u_in[c + 1];
        aw[0] += h0 * w_in[c];
        aw[1] += h1 * w_in[c + 1];
        if (!FIRST) {
          as[0] += h0 * s_in[c];
          as[1] += h1 * s_in[c + 1];
        }
        if (d == h) {
          hii[0] = h0;
          hii[1] = h1;
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        si[q] = FIRST ? 0.0 : s_in[ia + q];
        ui[q] = u_in[ia + q];
        wi[q] = w_in[ia + q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int i = q ? ib : ia;
        for_entries<S>(H, N, rw, i, [&](double hv, int k, bool diag) {
          ar[q] += hv * u_in[k];
          aw[q] += hv * w_in[k];
          if (!FIRST) as[q] += hv * s_in[k];
          if (diag) hii[q] = hv;
        });
        si[q] = FIRST ? 0.0 : s_in[i];
        ui[q] = u_in[i];
        wi[q] = w_in[i];
      }
    }
    if (!FIRST) {
      sc_rz = sc[kRZ];
      sc_alpha = sc[kAlpha];
      sc_bb = sc[kBB];
      sc_beta = sc[kBeta];
    }
    if constexpr (TOT) {
      acc[0] = part_in[4 * inst];
      acc[1] = part_in[4 * inst + 1];
      acc[2] = part_in[4 * inst + 2];
    } else {
      // the partials of the one-row kernel's threads 2t and 2t+1, each summed
      // in that kernel's order, then their pair sum
      double pa[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
      for (int q = 0; q < kTotBlocks / kBlock; ++q) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int b = 2 * t + v + q * kBlock;
          const double* pp = part_in + 4 * (b0 + min(b, nb - 1));
          const double wgt = b < nb ? 1.0 : 0.0;
          pa[v][0] += wgt * pp[0];
          pa[v][1] += wgt * pp[1];
          pa[v][2] += wgt * pp[2];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] = pa[0][k] + pa[1][k];
      pair_block_total<3>(acc, sh_in);
    }
  }
  // The values only the update needs (x, p and the previous residual, read
  // by launches of odd index) are requested after the stencil's arithmetic;
  // the barrier keeps the compiler from hoisting them.  Those launches then
  // fit four waves per SIMD with 7 diagonals (106 or 126 registers instead
  // of 152) and two with 19 (249 instead of 341).
  if constexpr (XW) {
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = q ? ib : ia;
      pld[q] = p_read ? p[i] : 0.0;
      uprev[q] = u_out[i];
      xold[q] = x[i];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 2; ++q) pld[q] = uprev[q] = xold[q] = 0.0;
  }
  const double gamma = acc[0], delta = acc[1], rr = acc[2];
  double alpha, beta, bb;
  if (FIRST) {
    bb = rr;
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    bb = sc_bb;
    beta = gamma / sc_rz;
    alpha = gamma / (delta - beta * gamma / sc_alpha);
  }
  double e_sum = 0.0, e_last = 0.0;
  const bool e_stop = !FIRST && stop.delay > 0 && energy_stop(sc, sc_alpha, sc_rz, it, stop, e_sum, e_last);
  int status = 0;
  if (!isfinite(rr)) status = 3;
  else if (rr <= stop.rtol2 * bb) status = 1;
  else if (e_stop) status = 1;
  else if (it >= stop.maxit) status = 2;
  else if (!isfinite(alpha) || !(alpha > 0.0)) status = 3;
  if (rw.bi == 0 && t == 0) {
    done[inst] = status;
    iters[inst] = it;
    double* so = scal_out + inst * kScal;
    so[kRZ] = gamma;
    so[kAlpha] = alpha;
    so[kBB] = bb;
    so[kBeta] = beta;
    if (stop.delay > 0) energy_record(sc, so, FIRST, it, stop.delay, e_sum, e_last);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) pold[q] = XW ? fma(sc_beta, pld[q], uprev[q]) : 0.0;   // p_{L-1}
  if (status != 0) {
    // the stop leaves x final (see k_cg_iter)
    if constexpr (XW) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (q ? vb : va) stream_store(&x[q ? ib : ia], fma(sc_alpha, pold[q], xold[q]));
    }
    if (t == 0) blk_done[L] = status;
    return;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) di[q] = 1.0 / hii[q];   // as the stored dinv was formed
  double sp[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double xn[2], pn[2], sn[2], un[2], wn[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double w_new = ar[q] - alpha * (aw[q] + beta * as[q]);
    pn[q] = fma(beta, pold[q], ui[q]);
    sn[q] = wi[q] + beta * si[q];
    xn[q] = fma(alpha, pn[q], fma(sc_alpha, pold[q], xold[q]));
    un[q] = ui[q] - alpha * sn[q];
    wn[q] = di[q] * w_new;
    const double rn = hii[q] * un[q];
    sp[q][0] = rn * un[q];
    sp[q][1] = w_new * un[q];
    sp[q][2] = rn * rn;
  }
  if (interior) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (XW) {
        stream_store(&x[ia + q], xn[q]);
        stream_store(&p[ia + q], pn[q]);
      }
      stream_store(&s_out[ia + q], sn[q]);
      stream_store(&u_out[ia + q], un[q]);
      stream_store(&w_out[ia + q], wn[q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (!(q ? vb : va)) {
        sp[q][0] = sp[q][1] = sp[q][2] = 0.0;
        continue;
      }
      const int i = q ? ib : ia;
      if (XW) {
        stream_store(&x[i], xn[q]);
        stream_store(&p[i], pn[q]);
      }
      stream_store(&s_out[i], sn[q]);
      stream_store(&u_out[i], un[q]);
      stream_store(&w_out[i], wn[q]);
    }
  }
  double tot[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) tot[k] = sp[0][k] + sp[1][k];
  pair_block_total<3>(tot, sh_out);
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) part_out[4 * L + k] = tot[k];
  }
}

// Post-solve update of node m (eq. final-sdc):
//   v_m += dv_m;  w_m += Gam_m + dt sum_{j<m} QE[m][j] dR_j;
//   (I_m, R_m) <- AP(v_m, w_m) with dI_m, dR_m their change;  amax = max(amax, |dv_m|).
template <int M, bool EMI, bool LIN>
__global__ __launch_bounds__(kBlock) void k_post(Map map, int m, int64_t N,
                                                 const double* __restrict__ ionic,
                                                 const double* __restrict__ x, double* v_m,
                                                 double* w_m, double* I_m, double* R_m,
                                                 double* dI_m, double* dR_m,
                                                 const double* __restrict__ Gam_m,
                                                 const double* __restrict__ dR, double* amax,
                                                 CollArgs c) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  const double d = x[i];
  if constexpr (EMI || LIN) {
    // potentials only; the sites (cell-by-cell) follow in k_post_sites, the
    // gating (linearized scheme) in k_wsweep after the last node
    v_m[i] += d;
    amax[i] = fmax(amax[i], fabs(d));
    return;
  }
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < M - 1; ++j)
    if (j < m) g += c.QE[m][j] * dR[j * N + i];
  const double vm = v_m[i] + d;
  const double wm = w_m[i] + (Gam_m[i] + c.dt * g);
  v_m[i] = vm;
  w_m[i] = wm;
  double In, Rn;
  ap_eval(vm, wm, ionic + 6 * rw.inst, In, Rn);
  dI_m[i] = In - I_m[i];
  dR_m[i] = Rn - R_m[i];
  I_m[i] = In;
  R_m[i] = Rn;
  amax[i] = fmax(amax[i], fabs(d));
}

// ---- the linearized scheme (the paper's basic scheme, eq. final-sdc)

// dR/dw of the Aliev-Panfilov rate: s (e_w g - e) with e = eps0 + mu1 w/(v + mu2),
// e_w = mu1 / (v + mu2), g = -w - k v (v - a - 1).
__device__ inline double ap_drdw(double v, double w, const double* p) {
  const double k = p[0], a = p[1], eps0 = p[2], mu1 = p[3], mu2 = p[4], s = p[5];
  const double e = eps0 + mu1 * w / (v + mu2);
  const double g = -w - k * v * (v - a - 1.0);
  return s * (mu1 / (v + mu2) * g - e);
}

// Sweep start of the linearized scheme: on the active rows, the lumped
// reaction Jacobian G_m = ML dI/dv(v_m, w_m) at the sweep's iterate, and the
// diagonal of every H_m = ML + dt QI[m][m] (A + G_m) (both storages, when
// present) with its Jacobi inverse.  Only the rows' own diagonals change,
// and a restricted solve reads no other row's diagonal.
template <int M>
__global__ __launch_bounds__(kBlock) void k_lin_diag(Map map, int64_t N, const double* __restrict__ ml,
                                                     const int32_t* __restrict__ diagpos,
                                                     const double* __restrict__ Aval,
                                                     const double* __restrict__ ionic,
                                                     const double* __restrict__ v, const double* __restrict__ w,
                                                     CollArgs c, double* __restrict__ G, double* __restrict__ Hval,
                                                     int64_t nnz, double* __restrict__ diaH, int64_t dstride,
                                                     double* __restrict__ dinv) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  const double* p = ionic + 6 * rw.inst;
  const double mli = ml[i];
  const int dg = diagpos[i];
  const double aii = Aval[dg];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double g = mli * ap_didv(v[m * N + i], w[m * N + i], p);
    const double cm = c.dt * c.QI[m][m];
    const double h = mli + cm * aii + cm * g;
    G[m * N + i] = g;
    Hval[m * nnz + dg] = h;
    if (diaH) diaH[m * dstride + i] = h;
    dinv[m * N + i] = 1.0 / h;
  }
}

// Gating of the linearized scheme after the potentials of all nodes
// (Gauss-Seidel, implicit dR/dw), per active row:
//   (1 - dt QI[m][m] R'_m) dw_m = w0 - w_m + dt sum_j Q[m][j] R(v_j, w_j) + dt sum_{j<m} QI[m][j] R'_j dw_j
// with R'_j = dR/dw(v_j, w_j) at the new potentials and the sweep's gating;
// then w_m += dw_m and (I_m, R_m) <- AP(v_m, w_m).
template <int M>
__global__ __launch_bounds__(kBlock) void k_wsweep(Map map, int64_t N, const double* __restrict__ ionic,
                                                   const double* __restrict__ v, double* __restrict__ w,
                                                   const double* __restrict__ w0, double* __restrict__ I,
                                                   double* __restrict__ R, CollArgs c) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  const double* p = ionic + 6 * rw.inst;
  double vj[M], wj[M], Rn[M], Rw[M], dw[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    vj[j] = v[j * N + i];
    wj[j] = w[j * N + i];
    double In;
    ap_eval(vj[j], wj[j], p, In, Rn[j]);
    Rw[j] = ap_drdw(vj[j], wj[j], p);
  }
  const double w0i = w0[i];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double sq = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) sq += c.Q[m][j] * Rn[j];
    double g = w0i - wj[m] + c.dt * sq;
#pragma unroll
    for (int j = 0; j < M; ++j)
      if (j < m) g += c.dt * c.QI[m][j] * Rw[j] * dw[j];
    dw[m] = g / (1.0 - c.dt * c.QI[m][m] * Rw[m]);
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double wm = wj[m] + dw[m];
    double In, Rm;
    ap_eval(vj[m], wm, p, In, Rm);
    w[m * N + i] = wm;
    I[m * N + i] = In;
    R[m * N + i] = Rm;
  }
}

// Cell-by-cell model, after k_post: the membrane sites whose intracellular
// node is active take the gating update and the new current and rate at the
// updated transmembrane voltage u_i - u_e.
template <int M>
__global__ __launch_bounds__(kBlock) void k_post_sites(Map map, int m, int64_t N,
                                                       const double* __restrict__ ionic, const double* v_m,
                                                       double* w_m, double* I_m, double* R_m, double* dI_m,
                                                       double* dR_m, const double* __restrict__ Gam_m,
                                                       const double* __restrict__ dR, CollArgs c, EmiArgs e) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
  if (!(e.sl[i] > 0.0)) return;
  double g = 0.0;
#pragma unroll
  for (int j = 0; j < M - 1; ++j)
    if (j < m) g += c.QE[m][j] * dR[j * N + i];
  const double wm = w_m[i] + (Gam_m[i] + c.dt * g);
  w_m[i] = wm;
  double In, Rn;
  ap_eval(v_m[i] - v_m[e.part[i]], wm, ionic + 6 * rw.inst, In, Rn);
  dI_m[i] = In - I_m[i];
  dR_m[i] = Rn - R_m[i];
  I_m[i] = In;
  R_m[i] = Rn;
}

// ---- active-set compaction (eq. "subset"): keep i with amax_i >= theta
// (keep_row in device.hpp).

// Pass 1: kept rows and their stored entries per block.
// theta: one drop tolerance, or (inst_theta not null) one per instance.
__global__ __launch_bounds__(kBlock) void k_select_count(Map map, const int32_t* __restrict__ rowptr,
                                                         const double* __restrict__ amax,
                                                         double theta, const double* __restrict__ inst_theta,
                                                         int32_t* sel_cnt, int32_t* sel_nnz,
                                                         const int32_t* __restrict__ stop) {
  __shared__ int sc[4], sn[4];
  const Row rw = map_row(map);
  if (rw.dead) return;
  const double th = inst_theta ? inst_theta[rw.inst] : theta;
  const bool keep = rw.valid && !(stop && stop[rw.inst]) && keep_row(amax[rw.row], th);
  const unsigned long long mask = __ballot(keep);
  int nz = keep ? rowptr[rw.row + 1] - rowptr[rw.row] : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nz += __shfl_xor(nz, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sc[wid] = __popcll(mask);
    sn[wid] = nz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sel_cnt[rw.blk] = sc[0] + sc[1] + sc[2] + sc[3];
    sel_nnz[rw.blk] = sn[0] + sn[1] + sn[2] + sn[3];
  }
}

constexpr int kScanThreads = 1024;

// Exclusive scan of one value per thread over a 1024-thread block.
__device__ int64_t block_exscan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

// In-place exclusive scan of a[0..n) (int32 or int64 values), one block.
template <class T>
__device__ int64_t scan_inplace(T* a, int n, int64_t* sh) {
  const int t = threadIdx.x;
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  int64_t s = 0;
  for (int q = lo; q < hi; ++q) s += a[q];
  int64_t total;
  int64_t run = block_exscan(s, sh, &total);
  for (int q = lo; q < hi; ++q) {
    const int64_t val = a[q];
    a[q] = static_cast<T>(run);
    run += val;
  }
  __syncthreads();
  return total;
}

// Fill a work map from per-instance counts and list offsets (one block).
// Returns false, with an empty map, when the counts need more entries than
// the record array holds (inconsistent counts: nothing is written past it).
__device__ bool build_map(const int32_t* cnt, const int32_t* aoff, int n_inst, const NextMap& nm,
                          int32_t total_rows) {
  __shared__ int fits;
  if (threadIdx.x == 0) {
    int64_t b = 0;
    for (int i = 0; i < n_inst; ++i) b += (static_cast<int64_t>(cnt[i]) + kBlock - 1) / kBlock;
    fits = b <= nm.cap;
    b = 0;
    for (int i = 0; i < n_inst; ++i) {
      const int32_t nb = fits ? (cnt[i] + kBlock - 1) / kBlock : 0;
      nm.inst_blk0[i] = static_cast<int32_t>(b);
      nm.inst_nblk[i] = nb;
      b += nb;
    }
    nm.totals[0] = static_cast<int32_t>(b);
    nm.totals[1] = fits ? total_rows : 0;
  }
  __syncthreads();
  const int32_t nblk = nm.totals[0];
  for (int b = threadIdx.x; b < nblk; b += kScanThreads) {
    int lo = 0, hi = n_inst - 1;   // last instance with inst_blk0 <= b
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (nm.inst_blk0[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const int bi = b - nm.inst_blk0[lo];
    BlkRec& r = nm.rec[b];
    r.inst = lo;
    r.beg = aoff[lo] + bi * kBlock;
    r.end = min(r.beg + kBlock, aoff[lo] + cnt[lo]);
    r.bi = bi;
    r.nb = nm.inst_nblk[lo];
    r.lo = static_cast<int32_t>(nm.node_off[lo]);
    r.hi = static_cast<int32_t>(nm.node_off[lo + 1]);
    r.pad = 0;
    for (int d = 0; d < nm.nd; ++d) r.off[d] = nm.dia_off[lo * nm.nd + d];
  }
  return fits;
}

// Pass 2 (one block): block offsets, per-instance totals, next work map.
__global__ __launch_bounds__(kScanThreads) void k_select_scan(Map map, int n_inst, int32_t* sel_cnt,
                                                              int32_t* sel_nnz, NextMap nm) {
  __shared__ int64_t sh[kScanThreads];
  int32_t* aoff_scratch = nm.aoff;
  // the entries the count pass covered: all of them, or those of the grid
  // when a live map outgrew it (entries past it hold an earlier scan's values)
  const int nb = min(map_entries(map), map.nblk);
  const int64_t total = scan_inplace<int32_t>(sel_cnt, nb, sh);
  const int64_t total_nnz = scan_inplace<int32_t>(sel_nnz, nb, sh);
  // an instance's blocks are consecutive: its totals are differences of the prefixes
  for (int i = threadIdx.x; i < n_inst; i += kScanThreads) {
    const int b0 = map.inst_blk0[i], b1 = b0 + map.inst_nblk[i];
    const int64_t c0 = b0 < nb ? sel_cnt[b0] : total, c1 = b1 < nb ? sel_cnt[b1] : total;
    const int64_t z0 = b0 < nb ? sel_nnz[b0] : total_nnz, z1 = b1 < nb ? sel_nnz[b1] : total_nnz;
    nm.inst_cnt[i] = static_cast<int32_t>(c1 - c0);
    nm.inst_nnz[i] = z1 - z0;
    aoff_scratch[i] = static_cast<int32_t>(c0);   // new list offset of instance i
  }
  if (threadIdx.x == 0) aoff_scratch[n_inst] = static_cast<int32_t>(total);
  __syncthreads();
  const bool fits = build_map(nm.inst_cnt, aoff_scratch, n_inst, nm, static_cast<int32_t>(total));
  if (threadIdx.x == 0) nm.totals[2] = fits ? 0 : 2;
}

// Pass 3: stable write of the kept rows; zero the work vectors on dropped rows.
// A kept row's list position q (over all instances) becomes position
// inst_blk0 * kBlock + (q - aoff) of its instance in the padded list.
__global__ __launch_bounds__(kBlock) void k_select_write(Map map, const double* __restrict__ amax,
                                                         double theta, const double* __restrict__ inst_theta,
                                                         const int32_t* __restrict__ sel_off, NextMap nm,
                                                         int32_t* __restrict__ idx_pad,
                                                         int32_t* __restrict__ idx_compact, ZeroVecs zv,
                                                         const int32_t* __restrict__ stop) {
  __shared__ int wc[4];
  const Row rw = map_row(map);
  if (rw.dead) return;
  const double th = inst_theta ? inst_theta[rw.inst] : theta;
  const bool keep = rw.valid && !(stop && stop[rw.inst]) && keep_row(amax[rw.row], th);
  const unsigned long long mask = __ballot(keep);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wc[wid] = __popcll(mask);
  __syncthreads();
  int base = sel_off[rw.blk];
  for (int q = 0; q < wid; ++q) base += wc[q];
  const int rank = __popcll(mask & ((1ull << lane) - 1ull));
  if (keep) {
    const int q = base + rank;
    const int64_t pos = static_cast<int64_t>(nm.inst_blk0[rw.inst]) * kBlock + (q - nm.aoff[rw.inst]);
    if (pos < static_cast<int64_t>(nm.inst_blk0[rw.inst] + nm.inst_nblk[rw.inst]) * kBlock) {
      idx_pad[pos] = rw.row;
      if (idx_compact) idx_compact[q] = rw.row;
    }
  }
  if (rw.valid && !keep && zv.dv) {
    const int i = rw.row;
#pragma unroll
    for (int q = 0; q < kZeroVecs; ++q) zv.vec[q][i] = 0.0;
    for (int m = 0; m < zv.M; ++m) zv.dv[m * zv.N + i] = 0.0;
    if (zv.dI)
      for (int m = 0; m < zv.M; ++m) {
        zv.dI[m * zv.N + i] = 0.0;
        zv.dR[m * zv.N + i] = 0.0;
      }
  }
}

__global__ __launch_bounds__(kBlock) void k_zero_rows(Map map, ZeroVecs zv) {
  const Row rw = map_row(map);
  if (!rw.valid) return;
  const int i = rw.row;
#pragma unroll
  for (int q = 0; q < kZeroVecs; ++q) zv.vec[q][i] = 0.0;
  for (int m = 0; m < zv.M; ++m) zv.dv[m * zv.N + i] = 0.0;
  if (zv.dI)
    for (int m = 0; m < zv.M; ++m) {
      zv.dI[m * zv.N + i] = 0.0;
      zv.dR[m * zv.N + i] = 0.0;
    }
}

// Work map of an ascending list, in three launches: k_list_prep clears the
// counters, k_list_scan validates the list and counts each instance's stored
// entries (one thread per entry), k_map_from_list (one block) finds the
// instances' ranges and builds the map.
__global__ __launch_bounds__(kBlock) void k_list_prep(int n_inst, NextMap nm) {
  for (int i = threadIdx.x; i < n_inst; i += kBlock) nm.inst_nnz[i] = 0;
  if (threadIdx.x == 0) nm.totals[2] = 0;
}

// Entry q is valid when it lies in [0, N) and above entry q - 1; any other
// entry marks the list invalid (totals[2] = 1, the same value from every
// writer).  A valid entry's row adds its stored entries of A to the count of
// its instance (the last i with node_off[i] <= row).  In a valid list the
// instances of a block's entries are consecutive: they are summed in LDS
// bins from the block's first instance and added with one atomic each
// (integer sums, so the order of the additions does not matter).
__global__ __launch_bounds__(kBlock) void k_list_scan(const int32_t* __restrict__ idx, int32_t n, int64_t N,
                                                      int n_inst, const int32_t* __restrict__ rowptr,
                                                      NextMap nm) {
  __shared__ unsigned long long bins[kBlock];
  __shared__ int first;
  const int q = static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
  bins[threadIdx.x] = 0;
  const bool live = q < n;
  const int32_t v = live ? idx[q] : 0;
  const bool ok = live && v >= 0 && v < N && (q == 0 || idx[q - 1] < v);
  if (live && !ok) nm.totals[2] = 1;
  int inst = -1;
  if (ok) {
    int lo = 0, hi = n_inst;   // node_off[lo] <= v < node_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nm.node_off[mid] <= v) lo = mid; else hi = mid;
    }
    inst = lo;
  }
  if (threadIdx.x == 0) first = inst;
  __syncthreads();
  const int k = inst - first;
  if (inst >= 0) {
    const auto z = static_cast<unsigned long long>(rowptr[v + 1] - rowptr[v]);
    if (first >= 0 && k >= 0 && k < kBlock) atomicAdd(&bins[k], z);
    else atomicAdd(reinterpret_cast<unsigned long long*>(&nm.inst_nnz[inst]), z);
  }
  __syncthreads();
  const int i = first + static_cast<int>(threadIdx.x);
  if (first >= 0 && i < n_inst && bins[threadIdx.x])
    atomicAdd(reinterpret_cast<unsigned long long*>(&nm.inst_nnz[i]), bins[threadIdx.x]);
}

// Instance i's entries of the list are those in [node_off[i],
// node_off[i+1]), found by binary search; then the map.  One block.  An
// invalid list (totals[2] from k_list_scan) gives an empty map and keeps
// totals[2] = 1, so no later kernel indexes with it.
__global__ __launch_bounds__(kScanThreads) void k_map_from_list(const int32_t* __restrict__ idx,
                                                                int32_t n, int n_inst, NextMap nm) {
  int32_t* aoff_scratch = nm.aoff;
  const int64_t* node_off = nm.node_off;
  const bool bad = nm.totals[2] != 0;
  if (bad) n = 0;
  for (int i = threadIdx.x; i <= n_inst; i += kScanThreads) {
    const int64_t key = node_off[i];
    int lo = 0, hi = n;   // first position with idx >= key
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (idx[mid] < key) lo = mid + 1; else hi = mid;
    }
    aoff_scratch[i] = lo;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_inst; i += kScanThreads) {
    nm.inst_cnt[i] = aoff_scratch[i + 1] - aoff_scratch[i];
    if (bad) nm.inst_nnz[i] = 0;
  }
  __syncthreads();
  const bool fits = build_map(nm.inst_cnt, aoff_scratch, n_inst, nm, n);
  if (threadIdx.x == 0) nm.totals[2] = bad ? 1 : fits ? 0 : 2;
}

// Energy of node m's correction on the map's rows: partial sums of x_i (H x)_i.
template <int S>
__global__ __launch_bounds__(kBlock) void k_energy(Map map, int64_t N, Mat H, const double* __restrict__ x,
                                                   double* __restrict__ e_part) {
  __shared__ double sh[16];
  const Row rw = map_row(map);
  if (rw.dead) return;
  double e[1] = {0.0};
  if (rw.valid) {
    const int i = rw.row;
    double hx = 0.0;
    for_entries<S>(H, N, rw, i, [&](double h, int k, bool) { hx += h * x[k]; });
    e[0] = x[i] * hx;
  }
  block_sum<1>(e, sh);
  if (threadIdx.x == 0) e_part[rw.blk] = e[0];
}

// One block per instance: energy over the M nodes and the stopping decision.
__global__ __launch_bounds__(kBlock) void k_energy_stop(const int32_t* __restrict__ inst_blk0,
                                                        const int32_t* __restrict__ inst_nblk, int M,
                                                        int64_t stride, const double* __restrict__ e_part,
                                                        double thr, int allow, double* __restrict__ energy,
                                                        int32_t* __restrict__ stop) {
  __shared__ double sh[16];
  const int inst = blockIdx.x, b0 = inst_blk0[inst], nb = inst_nblk[inst];
  double acc[1] = {0.0};
  for (int m = 0; m < M; ++m)
    for (int b = threadIdx.x; b < nb; b += kBlock) acc[0] += e_part[m * stride + b0 + b];
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) {
    energy[inst] = acc[0];
    if (allow && acc[0] <= thr) stop[inst] = 1;
  }
}

// ---- a-priori drop tolerance (Sec. 4.1, eq. drop-tolerance) after the first sweep

// Per block: the largest correction max_m |dv_m| (amax) of its rows, and the
// smallest dI/dv at the step's start state and at the collocation values.
template <int M>
__global__ __launch_bounds__(kBlock) void k_drop_part(Map map, int64_t N, const double* __restrict__ ionic,
                                                      const double* __restrict__ amax,
                                                      const double* __restrict__ v0,
                                                      const double* __restrict__ w0,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ part) {
  __shared__ double sh[8];
  const Row rw = map_row(map);
  if (rw.dead) return;
  double c = 0.0, d = INFINITY;
  if (rw.valid) {
    const int i = rw.row;
    const double* p = ionic + 6 * rw.inst;
    c = amax[i];
    d = ap_didv(v0[i], w0[i], p);
#pragma unroll
    for (int m = 0; m < M; ++m) d = fmin(d, ap_didv(v[m * N + i], w[m * N + i], p));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c = fmax(c, __shfl_xor(c, off, 64));
    d = fmin(d, __shfl_xor(d, off, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid] = c;
    sh[4 + wid] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * rw.blk] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    part[2 * rw.blk + 1] = fmin(fmin(sh[4], sh[5]), fmin(sh[6], sh[7]));
  }
}

// One block per instance: c = max |dv|, eta = max(0, -min dI/dv) (beta C_m = 1),
// r = the least r >= 0 with c rho^r <= (1 - rho) tol (Thm. 2, by repeated
// multiplication), TOL_drop = exp(-eta dt) (1 - rho) / (r + 1) tol.
// out[inst] = TOL_drop; info[4 inst ..] = (TOL_drop, r, c, eta).
__global__ __launch_bounds__(kBlock) void k_drop_tol(const int32_t* __restrict__ inst_blk0,
                                                     const int32_t* __restrict__ inst_nblk,
                                                     const double* __restrict__ part, double dt, double rho,
                                                     double tol, double* __restrict__ out,
                                                     double* __restrict__ info) {
  __shared__ double sh[8];
  const int inst = blockIdx.x, b0 = inst_blk0[inst], nb = inst_nblk[inst];
  double c = 0.0, d = INFINITY;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    c = fmax(c, part[2 * (b0 + b)]);
    d = fmin(d, part[2 * (b0 + b) + 1]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    c = fmax(c, __shfl_xor(c, off, 64));
    d = fmin(d, __shfl_xor(d, off, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid] = c;
    sh[4 + wid] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    d = fmin(fmin(sh[4], sh[5]), fmin(sh[6], sh[7]));
    const double eta = d < 0.0 ? -d : 0.0;   // also 0 for an instance without rows (d = inf)
    const double bound = (1.0 - rho) * tol;
    int r = 0;
    for (double q = c; q > bound && r < 10000; ++r) q *= rho;
    const double th = exp(-eta * dt) * (1.0 - rho) / (r + 1) * tol;
    out[inst] = th;
    info[4 * inst] = th;
    info[4 * inst + 1] = r;
    info[4 * inst + 2] = c;
    info[4 * inst + 3] = eta;
  }
}

// Copy of a list (validated by k_map_from_list) into the padded layout of its map.
__global__ __launch_bounds__(kBlock) void k_pad_list(const int32_t* __restrict__ idx, int32_t n, int n_inst,
                                                     NextMap nm, int32_t* __restrict__ idx_pad) {
  const int q = static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
  if (q >= n || nm.totals[2] != 0) return;
  int lo = 0, hi = n_inst - 1;   // last instance whose list starts at or before q
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nm.aoff[mid] <= q) lo = mid; else hi = mid - 1;
  }
  idx_pad[nm.inst_blk0[lo] * kBlock + (q - nm.aoff[lo])] = idx[q];
}

// The rows of a map as one list: entry b's rows go to positions beg..end.
__global__ __launch_bounds__(kBlock) void k_map_rows(Map map, int32_t* __restrict__ out) {
  const Row rw = map_row(map);
  if (rw.valid) out[rw.beg + static_cast<int>(threadIdx.x)] = rw.row;
}

inline dim3 grid(int nblk) { return dim3(static_cast<unsigned>(nblk > 0 ? nblk : 1)); }

// Whole restricted Jacobi-PCG of one instance in one workgroup (sets of at
// most kWgThreads * R rows): thread t owns list positions t + q kWgThreads,
// q < R.  R is a property of the matrix pattern (one row per thread for
// rows of more than 8 entries, whose unrolled loads need the 128 registers
// a wave of a 1024-thread workgroup has), so both storages of a matrix
// assign rows to threads alike and reduce in the same order.  Plain PCG with z = dinv r; the search direction
// is exchanged through pbuf (zero off the set, and everywhere again when the
// solve ends), with a workgroup barrier between its writes and the
// matrix-vector product that gathers it.  The reductions run in a fixed
// order (wave butterfly, then the waves in order), so every thread holds the
// same scalars and takes the same branches.
constexpr int kWgWaves = kWgThreads / 64;

template <int NV>
__device__ inline void wg_sum(double (&v)[NV], double* sh /* [kWgWaves * NV] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wid * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kWgWaves; ++q) a += sh[q * NV + k];
    v[k] = a;
  }
}

template <int S, int kWgRows>
__global__ __launch_bounds__(kWgThreads) void k_cg_wg(Map map, int64_t N, Mat H, const double* __restrict__ dinv,
                                                      const double* __restrict__ b, double* __restrict__ x,
                                                      double* __restrict__ pbuf, CgStop stop,
                                                      int32_t* __restrict__ done, int32_t* __restrict__ iters) {
  // one LDS array per reduction of an iteration, so that a reduction never
  // overwrites values another thread may still be reading
  __shared__ double sh_a[2 * kWgWaves], sh_b[kWgWaves], sh_c[2 * kWgWaves];
  // the energy-error stop's last step terms, t_j at ring[j % delay]; thread 0
  // writes the slot of step it after the barrier that follows the reads of
  // iteration it, and the reads of iteration it + 1 follow another barrier
  __shared__ double ring[kMaxDelay];
  const int inst = static_cast<int>(blockIdx.x);
  const int t = static_cast<int>(threadIdx.x);
  const int blk0 = map.inst_blk0[inst], nb = map.inst_nblk[inst];
  Row rw{};
  if (nb > 0) {
    // the instance's diagonal offsets and row range, from its first entry
    const int32_t* words = reinterpret_cast<const int32_t*>(map.rec + blk0);
    rw.word = words[min(t & 63, kRecWords - 1)];
    rw.lo = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, lo) / 4);
    rw.hi = __builtin_amdgcn_readlane(rw.word, offsetof(BlkRec, hi) / 4);
  }
  int row[kWgRows];
  bool valid[kWgRows];
  double xv[kWgRows], rv[kWgRows], pv[kWgRows], di[kWgRows];
  double acc[2] = {0.0, 0.0};   // r.z, b.b
#pragma unroll
  for (int q = 0; q < kWgRows; ++q) {
    const int pos = t + q * kWgThreads, e = pos / kBlock, lane = pos % kBlock;
    valid[q] = false;
    row[q] = 0;
    if (e < nb) {
      const BlkRec& rec = map.rec[blk0 + e];
      if (lane < rec.end - rec.beg) {
        valid[q] = true;
        row[q] = map.idx ? map.idx[(blk0 + e) * kBlock + lane] : rec.beg + lane;
      }
    }
    xv[q] = rv[q] = pv[q] = di[q] = 0.0;
    if (valid[q]) {
      const int i = row[q];
      rv[q] = b[i];
      di[q] = dinv[i];
      pv[q] = di[q] * rv[q];
      pbuf[i] = pv[q];
      acc[0] += rv[q] * pv[q];
      acc[1] += rv[q] * rv[q];
    }
  }
  wg_sum<2>(acc, sh_a);
  double rz = acc[0], rr = acc[1];
  const double bb = acc[1];
  int it = 0, status = 0;
  const int d = stop.delay;
  double e_sum = 0.0;   // sum_{j<it} t_j, t_j = alpha_j (r_j . z_j)
  for (;; ++it) {
    if (!isfinite(rr) || !isfinite(rz)) { status = 3; break; }
    if (rr <= stop.rtol2 * bb) { status = 1; break; }
    if (d > 0 && it >= d) {
      double win = 0.0;   // sum_{j=it-d}^{it-1} t_j, left to right
      for (int j = it - d; j < it; ++j) win += ring[j % d];
      if (win <= stop.etol2 * e_sum) { status = 1; break; }
    }
    if (it >= stop.maxit) { status = 2; break; }
    __syncthreads();   // pbuf holds the direction on every row of the set
    double qv[kWgRows];
    double pq[1] = {0.0};
#pragma unroll
    for (int q = 0; q < kWgRows; ++q) {
      qv[q] = 0.0;
      if (valid[q]) {
        double a = 0.0;
        for_entries<S>(H, N, rw, row[q], [&](double h, int k, bool) { a += h * pbuf[k]; });
        qv[q] = a;
        pq[0] += pv[q] * a;
      }
    }
    wg_sum<1>(pq, sh_b);
    if (!(pq[0] > 0.0)) { status = 3; break; }
    const double alpha = rz / pq[0];
    if (d > 0) {
      const double tj = alpha * rz;
      e_sum += tj;
      if (t == 0) ring[it % d] = tj;
    }
    double nr[2] = {0.0, 0.0};   // r.z, r.r after the update
#pragma unroll
    for (int q = 0; q < kWgRows; ++q) {
      if (valid[q]) {
        xv[q] += alpha * pv[q];
        rv[q] -= alpha * qv[q];
        const double z = di[q] * rv[q];
        nr[0] += rv[q] * z;
        nr[1] += rv[q] * rv[q];
      }
    }
    wg_sum<2>(nr, sh_c);
    const double beta = nr[0] / rz;
    rz = nr[0];
    rr = nr[1];
#pragma unroll
    for (int q = 0; q < kWgRows; ++q) {
      if (valid[q]) {
        pv[q] = di[q] * rv[q] + beta * pv[q];
        pbuf[row[q]] = pv[q];
      }
    }
  }
  __syncthreads();   // every gather of pbuf is done before it is cleared
#pragma unroll
  for (int q = 0; q < kWgRows; ++q) {
    if (valid[q]) {
      x[row[q]] = xv[q];
      pbuf[row[q]] = 0.0;
    }
  }
  if (t == 0) {
    done[inst] = status;
    iters[inst] = it;
  }
}

// The matrix-vector kernels outside the CG iteration (initial residual,
// energy) need few registers and run ~7-8 blocks per CU; on large maps
// their rows and the neighbour rows the stencil reaches (in 3D a plane
// away) then exceed the L2 and are fetched several times (128^3: 1.2 GB
// instead of 0.3 GB).  A dynamic LDS reservation caps such launches at 3
// blocks per CU.  The sweep kernels are register-limited already and lose
// time under the cap.
inline size_t cap_lds(const Map& map) { return map.nblk > 2048 ? 48 * 1024 : 0; }

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_spread(hipStream_t s, int M, const Map& all, int64_t N, const double* ionic,
                   const double* v0, const double* w0, double* v, double* w, double* I, double* R,
                   const EmiArgs& e) {
  if (all.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    constexpr int MM = decltype(mm)::value;
    if (e.part)
      k_spread<MM, true><<<grid(all.nblk), kBlock, 0, s>>>(all, N, ionic, v0, w0, v, w, I, R, e);
    else
      k_spread<MM, false><<<grid(all.nblk), kBlock, 0, s>>>(all, N, ionic, v0, w0, v, w, I, R, e);
  });
}

void launch_set_values(hipStream_t s, const int32_t* nodes, int64_t n, double value, double* v) {
  if (n <= 0) return;
  k_set_values<<<dim3(static_cast<unsigned>((n + 255) / 256)), 256, 0, s>>>(nodes, n, value, v);
}

void launch_sweep_start(hipStream_t s, int M, const Map& map, int64_t N, const Mat& A,
                        const double* ml, const double* v0, const double* w0, const double* v,
                        const double* w, const double* I, const double* R, double* Phi,
                        double* Gam, double* amax, const CollArgs& c, const EmiArgs& e) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    dispatch_storage(A, [&](auto st) {
      constexpr int MM = decltype(mm)::value, S = decltype(st)::value;
      if (e.part)
        k_sweep_start<MM, S, true><<<grid(map.nblk), kBlock, 0, s>>>(map, N, A, ml, v0, w0, v, w, I, R, Phi, Gam,
                                                                     amax, c, e);
      else
        k_sweep_start<MM, S, false><<<grid(map.nblk), kBlock, 0, s>>>(map, N, A, ml, v0, w0, v, w, I, R, Phi, Gam,
                                                                      amax, c, e);
    });
  });
}

void launch_rhs(hipStream_t s, int M, int m, const Map& map, int64_t N, const Mat& A,
                const double* ml, const double* Phi_m, const double* dI, const double* dv, double* r,
                double* x, const CollArgs& c, const EmiArgs& e, const double* G) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    dispatch_storage(A, [&](auto st) {
      constexpr int MM = decltype(mm)::value, S = decltype(st)::value;
      if (e.part)
        k_rhs<MM, S, true, false><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, A, ml, Phi_m, dI, dv, r, x, c, e,
                                                                    nullptr);
      else if (G)
        k_rhs<MM, S, false, true><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, A, ml, Phi_m, dI, dv, r, x, c, e, G);
      else
        k_rhs<MM, S, false, false><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, A, ml, Phi_m, dI, dv, r, x, c, e,
                                                                     nullptr);
    });
  });
}

void launch_lin_diag(hipStream_t s, int M, const Map& map, int64_t N, const double* ml, const int32_t* diagpos,
                     const double* Aval, const double* ionic, const double* v, const double* w, const CollArgs& c,
                     double* G, double* Hval, int64_t nnz, double* diaH, int64_t dstride, double* dinv) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    k_lin_diag<decltype(mm)::value><<<grid(map.nblk), kBlock, 0, s>>>(map, N, ml, diagpos, Aval, ionic, v, w, c, G,
                                                                      Hval, nnz, diaH, dstride, dinv);
  });
}

void launch_wsweep(hipStream_t s, int M, const Map& map, int64_t N, const double* ionic, const double* v,
                   double* w, const double* w0, double* I, double* R, const CollArgs& c) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    k_wsweep<decltype(mm)::value><<<grid(map.nblk), kBlock, 0, s>>>(map, N, ionic, v, w, w0, I, R, c);
  });
}

void launch_copy_b(hipStream_t s, const Map& map, const double* b, double* r, double* x) {
  if (map.nblk <= 0) return;
  k_copy_b<<<grid(map.nblk), kBlock, 0, s>>>(map, b, r, x);
}

void launch_cg_start(hipStream_t s, const Map& map, int n_inst, int64_t N, const Mat& H,
                     const double* dinv, const double* r0, double* u0, double* w0, double* part_out,
                     const CgState& cg) {
  const size_t lds = cap_lds(map);
  dispatch_storage(H, [&](auto st) {
    k_cg_start<decltype(st)::value><<<grid(map.nblk), kBlock, lds, s>>>(map, n_inst, N, H, dinv, r0, u0, w0,
                                                                        part_out, cg);
  });
}

bool compiled_diagonals(int nd) {
  bool fixed = false;
  dispatch_nd(nd, [&](auto st) { fixed = decltype(st)::value > 0; });
  return fixed;
}

void launch_cg_iter(hipStream_t s, const Map& map, int64_t N, const Mat& H, const double* dinv,
                    double* x, double* p, const double* u_in, const double* w_in, const double* s_in,
                    double* u_out, double* w_out, double* s_out, int it, const double* part_in,
                    double* part_out, const double* scal_in, double* scal_out, const CgStop& stop,
                    const CgState& cg, double* tot, bool pair_all, bool late, hipEvent_t ev_start,
                    hipEvent_t ev_stop) {
  if (map.nblk <= 0) return;
  const double* pin = part_in;
  late = late && tot && map.idx;   // listed sets: partial sums read late instead of the totals pass
  if (tot && !late) {
    k_cg_totals<<<dim3(static_cast<unsigned>(map.n_inst)), kBlock, 0, s>>>(map.inst_blk0, map.inst_nblk,
                                                                                 part_in, tot);
    pin = tot;
  }
  auto go = [&](auto kern, int threads) {
    if (ev_start) {
      // events stamped by the dispatch itself: they time the kernel's execution
      hipExtLaunchKernelGGL(kern, grid(map.nblk), dim3(threads), 0, s, ev_start, ev_stop, 0, cg.blk_done, map.rec,
                            map.idx, map.nblk, map.xcd_shift, map.live, it, pin, scal_in, N, H, dinv, x, p, u_in,
                            w_in, s_in, u_out, w_out, s_out, part_out, scal_out, stop, cg.done, cg.iters);
    } else {
      kern<<<grid(map.nblk), threads, 0, s>>>(cg.blk_done, map.rec, map.idx, map.nblk, map.xcd_shift, map.live, it,
                                              pin, scal_in, N, H, dinv, x, p, u_in, w_in, s_in, u_out, w_out, s_out,
                                              part_out, scal_out, stop, cg.done, cg.iters);
    }
  };
  // Launches of odd index write x (their own update and the one the launch
  // before deferred), launches of even index leave it: x is read and written
  // every other launch.
  dispatch_storage(H, [&](auto st) {
    constexpr int S = decltype(st)::value;
    auto pick = [&](auto tt, auto xw) {
      constexpr bool T = decltype(tt)::value, XW = decltype(xw)::value;
      if (map.idx && late) {
        it == 0 ? go(k_cg_iter<S, true, 1, 2, false>, kBlock) : go(k_cg_iter<S, false, 1, 2, XW>, kBlock);
      } else if (map.idx) {
        constexpr int TL = T ? 1 : 0;
        it == 0 ? go(k_cg_iter<S, true, 1, TL, false>, kBlock) : go(k_cg_iter<S, false, 1, TL, XW>, kBlock);
      } else if (S > 0 && pair_all) {
        // every row of the instances: two rows per thread
        if constexpr (S > 0)
          it == 0 ? go(k_cg_iter2<S, true, T, false>, kPairThreads) : go(k_cg_iter2<S, false, T, XW>, kPairThreads);
      } else {
        constexpr int TA = T ? 1 : 0;
        it == 0 ? go(k_cg_iter<S, true, 0, TA, false>, kBlock) : go(k_cg_iter<S, false, 0, TA, XW>, kBlock);
      }
    };
    const bool odd = (it & 1) != 0;
    if (tot)
      odd ? pick(std::true_type{}, std::true_type{}) : pick(std::true_type{}, std::false_type{});
    else
      odd ? pick(std::false_type{}, std::true_type{}) : pick(std::false_type{}, std::false_type{});
  });
}

void launch_post(hipStream_t s, int M, int m, const Map& map, int64_t N, const double* ionic,
                 const double* x, double* v_m, double* w_m, double* I_m, double* R_m,
                 double* dI_m, double* dR_m, const double* Gam_m, const double* dR, double* amax,
                 const CollArgs& c, const EmiArgs& e, bool lin) {
  if (map.nblk <= 0) return;
  dispatch_m(M, [&](auto mm) {
    constexpr int MM = decltype(mm)::value;
    if (e.part)
      k_post<MM, true, false><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, ionic, x, v_m, w_m, I_m, R_m, dI_m,
                                                                dR_m, Gam_m, dR, amax, c);
    else if (lin)
      k_post<MM, false, true><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, ionic, x, v_m, w_m, I_m, R_m, dI_m,
                                                                dR_m, Gam_m, dR, amax, c);
    else
      k_post<MM, false, false><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, ionic, x, v_m, w_m, I_m, R_m, dI_m,
                                                                 dR_m, Gam_m, dR, amax, c);
  });
}

void launch_post_sites(hipStream_t s, int M, int m, const Map& map, int64_t N, const double* ionic,
                       double* v_m, double* w_m, double* I_m, double* R_m, double* dI_m, double* dR_m,
                       const double* Gam_m, const double* dR, const CollArgs& c, const EmiArgs& e) {
  if (map.nblk <= 0 || !e.part) return;
  dispatch_m(M, [&](auto mm) {
    k_post_sites<decltype(mm)::value><<<grid(map.nblk), kBlock, 0, s>>>(map, m, N, ionic, v_m, w_m, I_m, R_m, dI_m,
                                                                        dR_m, Gam_m, dR, c, e);
  });
}

void launch_select(hipStream_t s, const Map& map, int n_inst, const int32_t* rowptr,
                   const double* amax, double theta, const double* inst_theta, int32_t* sel_cnt,
                   int32_t* sel_nnz, int32_t* idx_pad, int32_t* idx_compact, const NextMap& nm,
                   const ZeroVecs& zv, const int32_t* stop) {
  if (map.nblk > 0)
    k_select_count<<<grid(map.nblk), kBlock, 0, s>>>(map, rowptr, amax, theta, inst_theta, sel_cnt, sel_nnz,
                                                     stop);
  k_select_scan<<<1, kScanThreads, 0, s>>>(map, n_inst, sel_cnt, sel_nnz, nm);
  if (map.nblk > 0)
    k_select_write<<<grid(map.nblk), kBlock, 0, s>>>(map, amax, theta, inst_theta, sel_cnt, nm, idx_pad,
                                                     idx_compact, zv, stop);
}

void launch_drop_tolerance(hipStream_t s, const Map& map, int M, int64_t N, const double* ionic,
                           const double* amax, const double* v0, const double* w0, const double* v,
                           const double* w, double* part, double dt, double rho, double tol, double* out,
                           double* info) {
  if (map.nblk > 0)
    dispatch_m(M, [&](auto mm) {
      k_drop_part<decltype(mm)::value><<<grid(map.nblk), kBlock, 0, s>>>(map, N, ionic, amax, v0, w0, v, w, part);
    });
  k_drop_tol<<<dim3(static_cast<unsigned>(map.n_inst)), kBlock, 0, s>>>(map.inst_blk0, map.inst_nblk, part, dt, rho,
                                                                       tol, out, info);
}

void launch_cg_wg(hipStream_t s, const Map& map, int64_t N, const Mat& H, const double* dinv, const double* b,
                  double* x, double* pbuf, const CgStop& stop, const CgState& cg, int rows_per_thread) {
  if (map.n_inst <= 0) return;
  const dim3 g(static_cast<unsigned>(map.n_inst));
  dispatch_storage(H, [&](auto st) {
    constexpr int S = decltype(st)::value;
    if (rows_per_thread == 2)
      k_cg_wg<S, 2><<<g, kWgThreads, 0, s>>>(map, N, H, dinv, b, x, pbuf, stop, cg.done, cg.iters);
    else
      k_cg_wg<S, 1><<<g, kWgThreads, 0, s>>>(map, N, H, dinv, b, x, pbuf, stop, cg.done, cg.iters);
  });
}

void launch_energy(hipStream_t s, const Map& map, int64_t N, const Mat& H, const double* x, double* e_part) {
  if (map.nblk <= 0) return;
  dispatch_storage(H, [&](auto st) {
    k_energy<decltype(st)::value><<<grid(map.nblk), kBlock, cap_lds(map), s>>>(map, N, H, x, e_part);
  });
}

void launch_energy_stop(hipStream_t s, const Map& map, int M, int64_t stride, const double* e_part,
                        double thr, int allow, double* energy, int32_t* stop) {
  k_energy_stop<<<dim3(static_cast<unsigned>(map.n_inst)), kBlock, 0, s>>>(map.inst_blk0, map.inst_nblk, M, stride,
                                                                           e_part, thr, allow, energy, stop);
}

void launch_zero_rows(hipStream_t s, const Map& map, const ZeroVecs& zv) {
  if (map.nblk <= 0) return;
  k_zero_rows<<<grid(map.nblk), kBlock, 0, s>>>(map, zv);
}

void launch_map_from_list(hipStream_t s, const int32_t* idx, int64_t n, int64_t N, int n_inst,
                          const int32_t* rowptr, const NextMap& nm, int32_t* idx_pad) {
  k_list_prep<<<1, kBlock, 0, s>>>(n_inst, nm);
  if (n > 0)
    k_list_scan<<<dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
        idx, static_cast<int32_t>(n), N, n_inst, rowptr, nm);
  k_map_from_list<<<1, kScanThreads, 0, s>>>(idx, static_cast<int32_t>(n), n_inst, nm);
  if (n > 0)
    k_pad_list<<<dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
        idx, static_cast<int32_t>(n), n_inst, nm, idx_pad);
}

void launch_map_rows(hipStream_t s, const Map& map, int32_t* out) {
  if (map.nblk <= 0) return;
  k_map_rows<<<grid(map.nblk), kBlock, 0, s>>>(map, out);
}

}  // namespace sdc

namespace sdc {
namespace {
// H_m = ML + c_m A on the pattern of A, and dinv_m = 1 / diag(H_m).
// With the cell-by-cell model the membrane mass also has the partner entry.
__global__ __launch_bounds__(kBlock) void k_build_h(int64_t N, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ diagpos,
                                                    const double* __restrict__ A,
                                                    const double* __restrict__ ml, double c,
                                                    double* __restrict__ H, double* __restrict__ dinv,
                                                    const int32_t* __restrict__ ppos,
                                                    const double* __restrict__ pmass) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
  if (i >= N) return;
  const int dg = diagpos[i];
  const int pp = ppos ? ppos[i] : -1;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    // the diagonal in the same expression as the diagonal-storage build
    double h = (e == dg) ? ml[i] + c * A[e] : c * A[e];
    if (e == pp) h = pmass[i] + h;
    H[e] = h;
  }
  dinv[i] = 1.0 / H[dg];
}

__global__ void k_iota(int32_t* out, int64_t n) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t < n) out[t] = static_cast<int32_t>(t);
}
}  // namespace

void launch_build_h(hipStream_t s, int64_t N, const int32_t* rowptr, const int32_t* diagpos,
                    const double* A, const double* ml, double c, double* H, double* dinv,
                    const int32_t* ppos, const double* pmass) {
  k_build_h<<<dim3(static_cast<unsigned>((N + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
      N, rowptr, diagpos, A, ml, c, H, dinv, ppos, pmass);
}

namespace {
// Diagonal storage of H_m = ML + c A for the rows [lo, hi): the stored
// diagonal 0 is offset 0 and carries the mass (same expression as the CSR build).
__global__ __launch_bounds__(kBlock) void k_build_h_dia(int64_t N, int lo, int hi, int ns,
                                                        const double* __restrict__ A,
                                                        const double* __restrict__ ml, double c,
                                                        double* __restrict__ H) {
  const int i = lo + static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
  if (i >= hi) return;
  for (int d = 0; d < ns; ++d) {
    const int64_t q = d * N + i;
    H[q] = (d == 0) ? ml[i] + c * A[q] : c * A[q];
  }
}
}  // namespace

void launch_build_h_dia(hipStream_t s, int64_t N, int lo, int hi, int ns, const double* A,
                        const double* ml, double c, double* H) {
  if (hi <= lo) return;
  k_build_h_dia<<<dim3(static_cast<unsigned>((hi - lo + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
      N, lo, hi, ns, A, ml, c, H);
}

__global__ __launch_bounds__(kBlock) void k_build_sell(int64_t N, int nslice, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ sptr,
                                                       const double* __restrict__ val, double* __restrict__ sval) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= static_cast<int64_t>(nslice) * kSlice) return;
  const int sl = static_cast<int>(i / kSlice), lane = static_cast<int>(i % kSlice);
  const int e0 = sptr[sl], len = (sptr[sl + 1] - e0) / kSlice;
  const int n_row = i < N ? rowptr[i + 1] - rowptr[i] : 0;
  const int r0 = i < N ? rowptr[i] : 0;
  for (int d = 0; d < len; ++d) sval[e0 + d * kSlice + lane] = d < n_row ? val[r0 + d] : 0.0;
}

void launch_build_sell(hipStream_t s, int64_t N, int nslice, const int32_t* rowptr, const int32_t* sptr,
                       const double* val, double* sval) {
  const int64_t n = static_cast<int64_t>(nslice) * kSlice;
  k_build_sell<<<grid(static_cast<int>((n + kBlock - 1) / kBlock)), kBlock, 0, s>>>(N, nslice, rowptr, sptr, val,
                                                                                    sval);
}

void launch_iota(hipStream_t s, int32_t* out, int64_t n) {
  if (n <= 0) return;
  k_iota<<<dim3(static_cast<unsigned>((n + 255) / 256)), 256, 0, s>>>(out, n);
}

}  // namespace sdc
