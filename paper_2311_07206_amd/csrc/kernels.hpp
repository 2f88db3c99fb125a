// Launch interface of the device kernels (gfx950, wave64, FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdc {

constexpr int kBlock = 256;      // threads per block = active rows per block
constexpr int kMaxNodesDev = 6;  // collocation nodes supported by the kernels

// Collocation matrices and step length, passed by value (kernel arguments
// live in the scalar kernarg segment, read once per wave).
struct CollArgs {
  double Q[kMaxNodesDev][kMaxNodesDev];
  double QI[kMaxNodesDev][kMaxNodesDev];
  double QE[kMaxNodesDev][kMaxNodesDev];
  double dt;
};

constexpr int kRecDiag = 32;   // diagonal offsets held per block record

// Work map entry of one block.  The block processes kBlock consecutive
// positions [beg, end) of its instance's active list; `bi` is its index among
// that instance's blocks, which are consecutive entries of the map.  Every
// field depends only on the entry, so a kernel reads the record with the
// list entries of its rows in one round trip.
struct BlkRec {
  int32_t inst;
  int32_t beg, end;   // list positions; row numbers when the map has no list
  int32_t bi;
  int32_t nb;         // blocks of the instance
  int32_t lo, hi;     // the instance's rows [lo, hi)
  int32_t pad;
  int32_t off[kRecDiag];   // the instance's diagonal offsets (diagonal storage)
};

// Work map.  The list is stored padded by block: the rows of entry b are
// idx[b * kBlock + t] for t < end - beg (the tail of each block is unused).
// When idx is null the positions are row numbers (all rows active).
// live (graph-captured sweeps): the number of map entries, in device memory,
// written by the selection that built the map; the grid then has nblk >=
// *live blocks (the capacity), block b takes entry b and blocks past *live
// return at once.  Null: nblk is the number of entries (and the grid size).
// Order of a map's entries over the 8 XCDs: XCD x takes chunks of
// 2^xcd_shift consecutive entries, chunk c going to XCD c mod 8, and a tail
// shorter than 8 chunks in eighths.  kXcdContig makes every map one tail,
// i.e. each XCD a contiguous eighth.
constexpr int kXcdContig = 24;

struct Map {
  const BlkRec* rec;
  const int32_t* inst_blk0;   // first entry of each instance
  const int32_t* inst_nblk;   // entries of each instance
  const int32_t* idx;
  int32_t nblk;               // grid size
  int32_t n_inst;
  const int32_t* live = nullptr;
  int32_t xcd_shift = kXcdContig;
};

// Cell-by-cell model: membrane node pairs.  part[i] is the other node of
// node i's membrane site (-1: not a membrane node); sl[i] is the site's
// lumped membrane length, positive at the intracellular node (which holds
// the site's w, I, R), negative at the extracellular node, 0 elsewhere.  The
// membrane mass is cm |sl| on the diagonal and -cm |sl| at the partner; the
// ionic current enters node i as sl[i] * I(site).  part == null: monodomain.
struct EmiArgs {
  const int32_t* part;
  const double* sl;
  double cm;
};

struct Csr {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
};

// A matrix on the assembly pattern, stored either as CSR (nd == 0) or in
// symmetric diagonal storage: for instance i, entry d of row r lies in
// column r + off[i*nd + d] (offsets sorted, symmetric about 0, offset 0 at
// d = nd/2); the entries with offset o >= 0 are dval[(d - nd/2)*N + r], an
// entry with offset -o is read as the entry (r - o, r).  Entries absent from
// the pattern hold 0, and a column outside the instance is replaced by r
// itself (with value 0).
// With nd == 0 and sptr not null the entries are read from a sliced ELL copy
// instead of the CSR arrays: rows in slices of kSlice (one wavefront), slice
// s holding its entries column by column from sptr[s], entry d of row r at
// sptr[r / kSlice] + d * kSlice + r % kSlice, in the CSR order of the row and
// padded to the slice's longest row with value 0 in the row's own column
// (rowptr still gives each row's length).
struct Mat {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int32_t* off;
  const double* dval;
  const int64_t* node_off;
  int nd;
  const int32_t* sptr = nullptr;
  const int32_t* scol = nullptr;
  const double* sval = nullptr;
};
constexpr int kSlice = 64;

// Per-instance CG scalars, layout [n_inst][kScal] (one 128-byte line each).
// kRZ holds gamma = r.z; kE the running sum of the step terms alpha_j gamma_j
// and kRing.. the last kMaxDelay terms (term j at kRing + j % delay), kept
// for the energy-error stop.
enum { kRZ = 0, kBB, kAlpha, kBeta, kE, kRing = 8, kScal = 16 };
constexpr int kMaxDelay = kScal - kRing;

// Stopping rule of every CG solve.  The residual test ||r||^2 <= rtol2 ||b||^2;
// with delay d >= 1 also the energy-error test after update n >= d
//   sum_{j=n-d}^{n-1} t_j <= etol2 sum_{j<n} t_j,   t_j = alpha_j (r_j . z_j),
// (the last d terms estimate the squared energy error of x_{n-d}, the full sum
// is the squared energy of x_n, x0 = 0; Sec. 5.1 stops at an estimated
// energy-error reduction); maxit bounds the updates.
struct CgStop {
  double rtol2;
  double etol2;
  int maxit;
  int delay;   // 0: residual test only; 1..kMaxDelay
};

struct CgState {
  int32_t* done;       // per instance: 0 running, 1 converged, 2 maxit, 3 non-finite
  int32_t* iters;      // per instance: updates performed when the solve stopped
  int32_t* blk_done;   // per map entry: its instance's solve has stopped
};

void launch_spread(hipStream_t s, int M, const Map& all, int64_t N, const double* ionic,
                   const double* v0, const double* w0, double* v, double* w, double* I, double* R,
                   const EmiArgs& e);
void launch_set_values(hipStream_t s, const int32_t* nodes, int64_t n, double value, double* v);
void launch_sweep_start(hipStream_t s, int M, const Map& map, int64_t N, const Mat& A,
                        const double* ml, const double* v0, const double* w0, const double* v,
                        const double* w, const double* I, const double* R, double* Phi,
                        double* Gam, double* amax, const CollArgs& c, const EmiArgs& e);
// Right-hand side of node m; writes r = b and x = 0 on active rows.
void launch_rhs(hipStream_t s, int M, int m, const Map& map, int64_t N, const Mat& A,
                const double* ml, const double* Phi_m, const double* dI, const double* dv, double* r,
                double* x, const CollArgs& c, const EmiArgs& e,
                const double* G = nullptr);
void launch_copy_b(hipStream_t s, const Map& map, const double* b, double* r, double* x);
// Single-reduction Jacobi-PCG: start (w0 = H dinv r0 and partial sums), then
// one launch per iteration reading buffers (r, w, s)_in, writing (r, w, s)_out.
// Launch `it` reads the partial sums and scalars of launch it-1 (part_in,
// scal_in) and writes its own (part_out, scal_out); the start kernel's
// partials are the input of launch 0.  Every block sums its instance's
// partials itself unless `tot` is given ([n_inst][4] scratch): then a
// one-block-per-instance pass forms the totals first (for instances of more
// than kTotBlocks blocks, where the per-block sums would dominate).
// CG start from r0 = b: writes u0 = dinv b and dinv H u0 (the first
// iteration's u_in and w_in) and the partial sums.
void launch_cg_start(hipStream_t s, const Map& map, int n_inst, int64_t N, const Mat& H,
                     const double* dinv, const double* r0, double* u0, double* w0, double* part_out,
                     const CgState& cg);
// One CG launch; u, w, s are the preconditioner-scaled vectors dinv r,
// dinv H u and dinv H p (read from one buffer, written to the other).
// pair_all: maps without a list and diagonal storage take two rows per
// thread (else one); both give bitwise the same results.  compiled_diagonals:
// the diagonal count has a compile-time instantiation (3, 7, 19), where two
// rows per thread are available.
bool compiled_diagonals(int nd);
void launch_cg_iter(hipStream_t s, const Map& map, int64_t N, const Mat& H, const double* dinv,
                    double* x, double* p, const double* u_in, const double* w_in, const double* s_in,
                    double* u_out, double* w_out, double* s_out, int it, const double* part_in,
                    double* part_out, const double* scal_in, double* scal_out, const CgStop& stop,
                    const CgState& cg, double* tot, bool pair_all = true, bool late = false,
                    hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
constexpr int kTotBlocks = 4 * kBlock;
constexpr int kTotMapBlocks = 2048;
constexpr int kTotMinBlocks = 64;
// The whole restricted PCG of each instance in one workgroup of kWgThreads
// threads, rows_per_thread (1 or 2) rows each, for maps whose instances hold
// at most kWgThreads * rows_per_thread rows: x (zero on entry) receives the
// solution on the set, done/iters of cg the outcome; b is the right-hand
// side on the set; pbuf (double[N]) must be zero on entry and is zero again
// on return.  Plain PCG (z = dinv r) with the same stopping rules as the
// launch-per-iteration kernels.
constexpr int kWgThreads = 1024;
void launch_cg_wg(hipStream_t s, const Map& map, int64_t N, const Mat& H, const double* dinv, const double* b,
                  double* x, double* pbuf, const CgStop& stop, const CgState& cg, int rows_per_thread);
// Post-solve update of node m.  With the cell-by-cell model this updates the
// potentials and amax only; launch_post_sites then updates the membrane
// sites whose intracellular node is active, from the updated potentials.
void launch_post(hipStream_t s, int M, int m, const Map& map, int64_t N, const double* ionic,
                 const double* x, double* v_m, double* w_m, double* I_m, double* R_m,
                 double* dI_m, double* dR_m, const double* Gam_m, const double* dR, double* amax,
                 const CollArgs& c, const EmiArgs& e, bool lin = false);
// Linearized scheme (the paper's basic scheme): at the sweep start, G_m =
// ML dI/dv(v_m, w_m) and the diagonals of every H_m (CSR values, and the
// diagonal copy when diaH is not null; dstride = the copy's per-node stride)
// with dinv, on the map's rows; after the last node, the gating sweep.
void launch_lin_diag(hipStream_t s, int M, const Map& map, int64_t N, const double* ml, const int32_t* diagpos,
                     const double* Aval, const double* ionic, const double* v, const double* w, const CollArgs& c,
                     double* G, double* Hval, int64_t nnz, double* diaH, int64_t dstride, double* dinv);
void launch_wsweep(hipStream_t s, int M, const Map& map, int64_t N, const double* ionic, const double* v,
                   double* w, const double* w0, double* I, double* R, const CollArgs& c);
void launch_post_sites(hipStream_t s, int M, int m, const Map& map, int64_t N, const double* ionic,
                       double* v_m, double* w_m, double* I_m, double* R_m, double* dI_m, double* dR_m,
                       const double* Gam_m, const double* dR, const CollArgs& c, const EmiArgs& e);

// Active-set compaction I_{k+1} = {i in I_k : amax_i >= theta} (three passes).
// sel_cnt [nblk] and sel_nnz [nblk] are per-block scratch; next-map outputs
// and per-instance totals are written by the scan pass.  The block records
// take the instance ranges from node_off and, with diagonal storage (nd > 0),
// the instance's offsets from dia_off [n_inst][nd].
struct NextMap {
  BlkRec* rec;
  int32_t* inst_blk0;
  int32_t* inst_nblk;
  int32_t* inst_cnt;       // kept rows per instance
  int64_t* inst_nnz;       // stored A entries in kept rows per instance
  int32_t* aoff;           // [n_inst+1] compact list position of each instance's first row
  int32_t* totals;         // [0] total blocks, [1] total rows in the list, [2] invalid list
  const int64_t* node_off;
  const int32_t* dia_off;
  int nd;
  int32_t cap;             // entries rec (and cap * kBlock positions of the padded list) can hold
};
// Vectors that must be zero on inactive rows: the double-buffered CG vectors
// gathered at neighbouring columns (r, w, s) and the M node corrections dv[M][N].
constexpr int kZeroVecs = 6;
struct ZeroVecs {
  double* vec[kZeroVecs];
  double* dv;
  int M;
  int64_t N;
  // cell-by-cell model: the site changes dI, dR [M][N] of dropped sites
  // count as zero in later sweeps (null: monodomain)
  double* dI;
  double* dR;
};
// The kept rows are written to idx_pad (the padded list of the next map) and,
// when idx_compact is not null, also as one ascending list there.
// Rows of instances with stop[inst] != 0 (stop may be null) are dropped too.
void launch_select(hipStream_t s, const Map& map, int n_inst, const int32_t* rowptr,
                   const double* amax, double theta, const double* inst_theta, int32_t* sel_cnt,
                   int32_t* sel_nnz, int32_t* idx_pad, int32_t* idx_compact, const NextMap& nm,
                   const ZeroVecs& zv, const int32_t* stop);
// A-priori drop tolerance per instance from the first sweep on map (Sec. 4.1):
// out[inst] = TOL_drop, info[4 inst ..] = (TOL_drop, r, c, eta); part holds
// 2 doubles per map block.
void launch_drop_tolerance(hipStream_t s, const Map& map, int M, int64_t N, const double* ionic,
                           const double* amax, const double* v0, const double* w0, const double* v,
                           const double* w, double* part, double dt, double rho, double tol, double* out,
                           double* info);
// Energy-norm termination (Sec. 3.2): per block of the map, the partial sum
// of x_i (H x)_i over its rows -> e_part[block]; then, per instance, the sum
// over the M nodes' partials (node-major, blocks in order) -> energy[inst],
// and stop[inst] |= allow && energy <= thr.
void launch_energy(hipStream_t s, const Map& map, int64_t N, const Mat& H, const double* x, double* e_part);
void launch_energy_stop(hipStream_t s, const Map& map, int M, int64_t stride, const double* e_part,
                        double thr, int allow, double* energy, int32_t* stop);
// Zero the ZeroVecs entries on every row of the map (used before a pinned set).
void launch_zero_rows(hipStream_t s, const Map& map, const ZeroVecs& zv);
// Work map of an arbitrary ascending list (per-instance split by node_off),
// with the list copied padded to idx_pad.  A list with entries outside
// [0, N) or not strictly ascending yields an empty map and totals[2] = 1.
void launch_map_from_list(hipStream_t s, const int32_t* idx, int64_t n, int64_t N, int n_inst,
                          const int32_t* rowptr, const NextMap& nm, int32_t* idx_pad);
// The rows of a map as one ascending list (list positions beg..end of each entry).
void launch_map_rows(hipStream_t s, const Map& map, int32_t* out);

// Heuristic first-sweep set (subset.hip): mark[0..n) = 0; mark[rows[q]] = 1
// (rows in [0, n)); one ring of growth out_i = max of in over row i's pattern.
void launch_mark_clear(hipStream_t s, double* mark, int64_t n);
void launch_mark_rows(hipStream_t s, const int32_t* rows, int64_t n, double* mark);
void launch_mark_grow(hipStream_t s, const int32_t* rowptr, const int32_t* col, const double* in, double* out,
                      int64_t n);

// H_m = ML + c A (pattern of A) and its inverse diagonal.
// ppos[i] (or null): CSR position of node i's membrane partner column (-1:
// none), where pmass[i] is added (the off-diagonal membrane mass).
void launch_build_h(hipStream_t s, int64_t N, const int32_t* rowptr, const int32_t* diagpos,
                    const double* A, const double* ml, double c, double* H, double* dinv,
                    const int32_t* ppos, const double* pmass);
void launch_iota(hipStream_t s, int32_t* out, int64_t n);
// Sliced ELL values from CSR values on the same pattern: sval[sptr[r / kSlice]
// + d * kSlice + r % kSlice] = val[rowptr[r] + d] for d below row r's length,
// 0 for the padding (nslice slices, N rows).
void launch_build_sell(hipStream_t s, int64_t N, int nslice, const int32_t* rowptr, const int32_t* sptr,
                       const double* val, double* sval);
// Diagonal storage of H_m = ML + c A for the rows [lo, hi): ns stored
// diagonals, the first of which is offset 0.
void launch_build_h_dia(hipStream_t s, int64_t N, int lo, int hi, int ns, const double* A,
                        const double* ml, double c, double* H);

// ---- reverse (adjoint) step; see adjoint_kernels.hip for the equations
void launch_adj_sweep_init(hipStream_t s, int M, const Map& map, int64_t N, const double* Lv,
                           const double* Lw, double* Ldv, double* Ldw);
void launch_adj_dw(hipStream_t s, int M, int m, const Map& map, int64_t N, const double* ionic,
                   const double* V, const double* W, const double* Ve, const double* We, double* Lv,
                   double* Lw, double* Ldv, double* Ldw, double* Lw0, double* ga_row, const CollArgs& c);
void launch_adj_apsi(hipStream_t s, int M, int m, const Map& all, int64_t N, const Mat& A,
                     const double* ml, const double* ionic, const uint8_t* in_set, const double* psi,
                     const double* V, const double* W, const double* Ve, const double* We,
                     const double* DV, double* Lv, double* Lw, double* Ldv, double* Ldw, double* Lv0,
                     double* ga_row, double* u, const CollArgs& c);
void launch_adj_elem(hipStream_t s, int nv, int64_t ne, const int32_t* elems, const double* pairw,
                     const double* psi, const double* u, double* qe);
void launch_adj_spread(hipStream_t s, int M, int64_t N, const double* Lv, const double* Lw, double* Lv0,
                       double* Lw0);
void launch_adj_gather_sigma(hipStream_t s, int64_t N, int nv, const int32_t* nptr, const int32_t* nel,
                             const double* qe, double* g);
void launch_adj_reduce_a(hipStream_t s, int n_inst, const int64_t* node_off, const double* ga_row, double* g_a);
void launch_set_flags(hipStream_t s, const Map& map, uint8_t* flags, uint8_t value);
void launch_zero_values(hipStream_t s, const int32_t* nodes, int64_t n, double* v);

}  // namespace sdc
