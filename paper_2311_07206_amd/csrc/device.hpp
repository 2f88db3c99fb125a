// Device helpers shared by the forward and reverse kernels: block order and
// the row a thread owns in a work map.
#pragma once

#include "kernels.hpp"

namespace sdc {

// The drop rule of the active sets (eq. "subset"): a row stays when its
// largest correction reached the drop tolerance; theta <= 0 keeps every row
// (the non-adaptive method); NaN is dropped otherwise.
__device__ inline bool keep_row(double a, double theta) { return theta <= 0.0 || a >= theta; }

constexpr int kRecWords = static_cast<int>(sizeof(BlkRec) / sizeof(int32_t));

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8).  Give each XCD runs of consecutive map entries instead, so that
// neighbouring row blocks, which read each other's rows through the stencil,
// share one L2: XCD x takes chunks x, x + 8, x + 16, ... of 2^sh entries (in
// order), and the entries past the last full round of 8 chunks in contiguous
// eighths.  Chunks a few times the stencil's reach keep the reads inside one
// L2 and still deal every XCD an even share of a batch's instances, also when
// some of them have stopped iterating (contiguous eighths would leave the
// XCDs whose eighth holds stopped instances idle).  A bijection of [0, nblk)
// when the grid has nblk workgroups.
__device__ inline int logical_block(int nblk, int sh) {
  const int b = static_cast<int>(blockIdx.x);
  const int x = b & 7, k = b >> 3;
  const int full = (nblk >> (sh + 3)) << (sh + 3);   // entries in full rounds of 8 chunks
  if (b < full) return ((((k >> sh) << 3) + x) << sh) + (k & ((1 << sh) - 1));
  const int n = nblk - full, q = n >> 3, rem = n & 7;
  return full + x * q + min(x, rem) + ((b - full) >> 3);
}

// The thread's row and its block's map entry.  Each wave reads the entry with
// one vector load (lane q holds word q) and takes the fields from the lanes:
// vector loads complete in order, so the entry and the list entry of the row
// (at a position known from the block index alone) arrive in one round trip.
// With a live count in device memory (graph-captured sweeps) the grid is
// the map's capacity: the XCD order is taken over the grid (a bijection of
// it, so every live entry gets a block), the count arrives in the same round
// trip, and `dead` marks blocks whose entry lies past it.
struct Row {
  int word;   // word (lane mod kRecWords) of the block record
  int inst, beg, end, bi, nb, lo, hi;
  int listed; // the list entry at the thread's position (0 without a list)
  int row;
  int blk;    // logical block: position of the entry in the map
  bool valid;
  bool dead;  // a block past the live entries: returns without writing
  // diagonal offset d of the instance (uniform d)
  __device__ int off(int d) const { return __builtin_amdgcn_readlane(word, offsetof(BlkRec, off) / 4 + d); }
};

// The number of entries of a map (a device load when it is live).
__device__ inline int map_entries(const Map& map) { return map.live ? *map.live : map.nblk; }

// LIST: 1 the map has a list, 0 all rows, -1 decided at run time.
template <int LIST = -1>
__device__ inline Row map_row(const Map& map) {
  const int L = logical_block(map.nblk, map.xcd_shift);
  const int t = static_cast<int>(threadIdx.x);
  const int32_t* words = reinterpret_cast<const int32_t*>(map.rec + L);
  Row r;
  r.word = words[min(t & 63, kRecWords - 1)];
  r.listed = 0;
  if (LIST == 1 || (LIST < 0 && map.idx)) r.listed = map.idx[L * kBlock + t];
  const int n_live = map.live ? *map.live : map.nblk;
  r.inst = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, inst) / 4);
  r.beg = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, beg) / 4);
  r.end = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, end) / 4);
  r.bi = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, bi) / 4);
  r.nb = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, nb) / 4);
  r.lo = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, lo) / 4);
  r.hi = __builtin_amdgcn_readlane(r.word, offsetof(BlkRec, hi) / 4);
  r.blk = L;
  r.dead = L >= n_live;
  r.valid = !r.dead && t < r.end - r.beg;
  const bool listed_map = LIST == 1 || (LIST < 0 && map.idx);
  r.row = r.valid ? (listed_map ? r.listed : r.beg + t) : 0;
  return r;
}

}  // namespace sdc
