// fg_sat.h -- state of the spatial-approximation-tree forest builder.
#pragma once
#include <vector>
#include "fg_internal.h"

namespace fg {

constexpr int kSmall = 1024;  // bags up to this size are built by one wave

// A bag: the not-yet-placed descendants of node `center` in tree t, at
// positions [start, start + len) of the position space.  pos / nN / nN_prev
// track the acceptance walk of a large bag.
struct SatSeg {
  uint32_t t, center;
  uint64_t start;
  uint32_t len, pos, nN, nN_prev;
};

struct SatTile {
  uint32_t seg, off;  // kTile positions of segment `seg` from offset `off`
};

struct SatCtl {
  unsigned long long counters[3];  // key distances, acceptance tests, assignment
  uint32_t active, n_next, n_small;
  int status;                      // bit 3: a segment list overflowed
};

struct SatArgs {
  RowSet X;
  int64_t n;
  uint32_t* perm;
  uint32_t* perm2;
  uint64_t* key;
  uint8_t* flag;     // 0 undecided, 1 neighbour, 2 rejected
  uint32_t* owner;   // child index of a rejected candidate
  uint32_t* nl;      // neighbour lists of the large bags (at the bag's start)
  uint32_t* ccount;  // per child: bag size, then scatter cursor
  uint32_t* coff;    // per child: bag offset
  uint32_t *stk_a, *stk_s, *stk_m, *stk_tmp;
  uint32_t* parent;  // T x n
  SatSeg* segs;
  SatSeg* next;
  uint32_t cap_next;
  SatSeg* small;
  uint32_t cap_small;
  SatTile* tiles;
  unsigned long long* counters;
  uint32_t* active;
  uint32_t* n_next;
  uint32_t* n_small;
  int* status;
  // float32 rows of more than 256 elements: |x_i|^2 of every row (any
  // float32 summation order), for the matrix-core closest-neighbour
  // assignment (NULL: exact streaming assignment only)
  const float* norm;
  int d;
  // batched builds: each id's instance and the 16-byte chunks of that
  // instance's own rows (NULL: every row has X.Q chunks)
  const uint16_t* inst_of;
  const int* inst_q;
};

struct SatWs {
  size_t perm, perm2, key, key2, flag, owner, nl, ccount, coff, stk_a, stk_s, stk_m, stk_tmp;
  size_t segs, next, small, tiles, ctl, norm, total;
  uint32_t cap_segs, cap_small, cap_tiles;
};

size_t sat_workspace_bytes(int64_t n, uint32_t T, SatWs* w);
// Build T trees rooted at roots (device); parent is T x n (device).
hipError_t sat_build(const Shape& s, const uint32_t* roots, uint32_t T, uint32_t* parent, char* ws,
                     const SatWs& w, hipStream_t st, unsigned long long* evals, int* status);
// The trees of several instances at once: instance i owns the ids
// [off, off + n) of s (rows of other instances are never compared with
// them) and its trees are rooted at off + roots[t] (roots: host, local ids,
// T <= 64).  parent is T x s.n in the shared ids; ids of no instance keep
// 0xFFFFFFFF.  Every instance gets exactly the trees of its own build.
struct SatInstance {
  int64_t off, n;
  const uint32_t* roots;
};
// inst_of / inst_q (optional, device): each id's instance and the chunks of
// its own rows, so that bags read only those.
hipError_t sat_build_multi(const Shape& s, uint32_t T, const std::vector<SatInstance>& inst, uint32_t* parent,
                           char* ws, const SatWs& w, hipStream_t st, unsigned long long* evals, int* status,
                           const uint16_t* inst_of = nullptr, const int* inst_q = nullptr);
// Directed edges of the T trees in both directions, grouped by source row
// (unsorted, with repeats) into tmp_ids at offsets off_tmp.
hipError_t tree_edges_csr(int64_t n, uint32_t T, const uint32_t* parent, uint32_t* deg,
                          uint64_t* off_tmp, uint32_t* cursor, uint32_t* tmp_ids, hipStream_t st,
                          void* scan_scratch);

}  // namespace fg
