// fg_sat.hip -- the scaffold S_0 (Sec. 1, Sec. 3): T classic spatial-
// approximation trees (Navarro 2002) built together, and the union of their
// edges in both directions.
//
// A node a with bag S: sort S by (d(v,a), id); walking that order, v becomes
// a neighbour of a iff d(v,a) < d(v,b) for every neighbour b accepted
// before it; every other v joins the bag of its closest neighbour (ties by
// the neighbour's id).  Rejection of v by b is d(v,b) <= d(v,a): exactly the
// occlusion prune with alpha = 1 and no degree bound, so acceptance reuses
// prune_wave().
//
// Layout: position space [0, T*n), tree t owning [t*n, (t+1)*n).  Every bag
// is a contiguous range of `perm`; after a node is processed its range holds
// its neighbours (in acceptance order) followed by their bags.
//
//   large bags (> kSmall points): level-synchronous passes over all trees --
//     distances to the node, segmented sort (wave tile sort + merge passes),
//     acceptance in chunks of 64 candidates (one wave per bag) interleaved
//     with a filter pass that rejects the remaining candidates against the
//     chunk's new neighbours, closest-neighbour assignment, partition;
//   small bags: one wave builds the whole subtree with an explicit stack.
#include <algorithm>
#include <vector>

#include "fg_sat.h"

namespace fg {

namespace {

constexpr int kTile = 256;  // positions per wave in the large-bag passes

// The rows a bag centred at `center` compares: in a batched build only the
// chunks of the instance's own rows (the padding is zero and adds exactly
// nothing).  Rows of more than 64 chunks keep the full length.
template <int NCH>
__device__ __forceinline__ RowSet sat_rows(const SatArgs& A, uint32_t center) {
  RowSet X = A.X;
  if constexpr (NCH <= 4)
    if (A.inst_q) X.Q = A.inst_q[A.inst_of[center]];
  return X;
}

// ---------------------------------------------------------------- large bags
// Keys (d(v, center), v) of every position of the large bags.
template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_sat_keys(SatArgs A) {
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  const int lane = lane_id(), g = lane % L;
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  Chunks<L, NCH> ac;
  const RowSet X = sat_rows<NCH>(A, sg.center);
  load_chunks<L, NCH>(ac, X.x + (size_t)sg.center * X.stride, X.Q, g);
  uint32_t an = 0;
  if constexpr (DK == U8L2) an = group_sum_u32<L>(u8_selfdot<L, NCH>(ac));
  const uint32_t lo = tl.off, hi = min(sg.len, tl.off + kTile);
  for (uint32_t base = lo; base < hi; base += 64) {
    int cnt = (int)min(64u, hi - base);
    if (lane < cnt) cid[lane] = A.perm[sg.start + base + lane];
    wave_sync();
    batch_dists_rs<DK, L, NCH>(X, ac, an, cid, cnt, ckey);
    if (lane < cnt) {
      A.key[sg.start + base + lane] = ckey[lane];
      A.flag[sg.start + base + lane] = 0;
    }
    wave_sync();
  }
  if (lane == 0) atomicAdd(&A.counters[0], (unsigned long long)(hi - lo));
}

// Sort each tile of kTile keys (tiles never straddle a bag).
__global__ void __launch_bounds__(64) k_sat_tile_sort(SatArgs A) {
  __shared__ uint64_t sk[kTile];
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint32_t cnt = min((uint32_t)kTile, sg.len - tl.off);
  for (int i = lane; i < kTile; i += 64) sk[i] = i < (int)cnt ? A.key[sg.start + tl.off + i] : FG_KEY_NONE;
  wave_sync();
  wave_sort_lds<uint64_t>(sk, kTile);
  for (int i = lane; i < (int)cnt; i += 64) A.key[sg.start + tl.off + i] = sk[i];
}

// One merge pass: runs of width w (sorted) pairwise merged from src to dst.
__global__ void __launch_bounds__(64) k_sat_merge_pass(SatArgs A, const uint64_t* src, uint64_t* dst,
                                                       uint32_t w) {
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint64_t* s = src + sg.start;
  uint64_t* d = dst + sg.start;
  const uint32_t hi = min(sg.len, tl.off + kTile);
  for (uint32_t j = tl.off + lane; j < hi; j += 64) {
    uint64_t k = s[j];
    uint32_t r = j / w;
    uint32_t pb = (r & ~1u) * w;  // pair base
    uint32_t other_lo, other_hi, mine;
    if ((r & 1u) == 0) {
      mine = j - pb;
      other_lo = min(pb + w, sg.len);
      other_hi = min(pb + 2 * w, sg.len);
    } else {
      mine = j - pb - w;
      other_lo = pb;
      other_hi = pb + w;
    }
    // stable: the left run's keys go before equal keys of the right run
    const bool left = (r & 1u) == 0;
    uint32_t a = other_lo, b = other_hi;
    while (a < b) {
      uint32_t m = (a + b) >> 1;
      if (left ? (s[m] < k) : (s[m] <= k)) a = m + 1;
      else b = m;
    }
    d[pb + mine + (a - other_lo)] = k;
  }
}

// After sorting: perm follows the keys.
__global__ void __launch_bounds__(64) k_sat_perm_from_keys(SatArgs A) {
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kTile);
  for (uint32_t j = tl.off + lane; j < hi; j += 64) A.perm[sg.start + j] = key_id(A.key[sg.start + j]);
}

// One wave per large bag: the next (up to) 64 undecided candidates after
// `pos`, in key order, resolved among themselves; accepted ones are
// appended to the bag's neighbour list.
template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_sat_resolve(SatArgs A) {
  __shared__ uint64_t sk[64];
  __shared__ uint32_t alive[2];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  __shared__ uint32_t acc[64];
  const int lane = lane_id();
  SatSeg* sgp = &A.segs[blockIdx.x];
  SatSeg sg = *sgp;
  sg.nN_prev = sg.nN;
  if (sg.pos >= sg.len) {
    if (lane == 0) sgp->nN_prev = sg.nN;
    return;
  }
  int k = 0;
  uint32_t pos = sg.pos;
  while (pos < sg.len && k < 64) {
    uint32_t j = pos + lane;
    bool und = j < sg.len && A.flag[sg.start + j] == 0;
    uint64_t m = ballot(und);
    int take = min(popc64(m), 64 - k);
    int rank = popc64(m & lanes_below());
    if (und && rank < take) sk[k + rank] = A.key[sg.start + j];
    // positions up to the last taken one are consumed
    if (take < popc64(m)) {
      // find the lane of the take-th undecided entry
      uint64_t mm = m;
      for (int t = 0; t < take; t++) mm &= mm - 1;
      int stop = __ffsll((long long)mm) - 1;
      pos += stop;
    } else {
      pos = min(pos + 64, sg.len);
    }
    k += take;
  }
  wave_sync();
  unsigned long long pe = 0;
  int kept = prune_wave<DK, L, NCH>(sat_rows<NCH>(A, sg.center), 1.0f, 65, sk, k, alive, cid, ckey, acc, &pe);
  // prune_wave left alive bits on exactly the accepted candidates.  Mark
  // the chunk's positions: they are the first k undecided ones from the old
  // pos, so walk them again in the same order.
  {
    uint32_t p2 = sg.pos;
    int seen = 0;
    while (seen < k) {
      uint32_t j = p2 + lane;
      bool und = j < sg.len && A.flag[sg.start + j] == 0;
      uint64_t m = ballot(und);
      int rank = popc64(m & lanes_below());
      if (und && seen + rank < k) {
        int i = seen + rank;
        bool a = (alive[i >> 5] >> (i & 31)) & 1u;
        A.flag[sg.start + j] = a ? 1 : 2;
      }
      seen += popc64(m);
      p2 += 64;
    }
  }
  for (int i = lane; i < kept; i += 64) A.nl[sg.start + sg.nN + i] = acc[i];
  if (lane == 0) {
    sgp->nN_prev = sg.nN;
    sgp->nN = sg.nN + kept;
    sgp->pos = pos;
    if (pos < sg.len) atomicAdd(A.active, 1u);
    atomicAdd(&A.counters[1], pe);
  }
}

// The filter's tests for float32 rows of more than 64 chunks: the cnt
// candidates (ids in key order of cdk, positions cpos) against the nb new
// neighbours from 32x32 matrix-core tiles with the Gram-tile prune's margin.
// A test is decided from d~ when the margin allows (reject when fl(d~ + eps)
// <= d(v,a), keep when fl(d~ - eps) > d(v,a)), else from the exact
// declared-order distance; each candidate walks the neighbours in acceptance
// order to its first rejection, so flags and the test count are those of the
// exact loop.  dec: LDS [64 * 64] decision codes.
template <int DK, int L, int NCH>
__device__ void filter_gram(const SatArgs& A, const SatSeg& sg, int cnt, const uint32_t* nbr, int nb,
                            const uint32_t* cpos, const uint64_t* cdk, uint8_t* dec, uint32_t* qv,
                            uint32_t* qb, float* qd, unsigned long long* ev) {
  constexpr int G = 64 / L;
  constexpr uint8_t KEEP = 0, REJ = 1, UNSURE = 2;
  const int lane = lane_id(), h = lane >> 5, g = lane % L;
  const float u8 = 8.0f * 5.9604645e-08f;
  const RowSet& X = A.X;
  for (int I = 0; 32 * I < cnt; I++) {
    const int ra = 32 * I + (lane & 31);
    const uint8_t* pa = X.x + (size_t)key_id(cdk[ra < cnt ? ra : 0]) * X.stride + 16 * h;
    float na[16], dva[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int i = 32 * I + gram_acc_row(r, lane);
      const uint64_t k = cdk[i < cnt ? i : 0];
      na[r] = A.norm[key_id(k)];
      dva[r] = hi_to_float<DK>(key_hi(k));
    }
    for (int J = 0; 32 * J < nb; J++) {
      const int jb = 32 * J + (lane & 31);
      const uint32_t b = nbr[jb < nb ? jb : 0];
      const float nbn = A.norm[b];
      gram_f32x16 acc;
#pragma unroll
      for (int e = 0; e < 16; e++) acc[e] = 0.0f;
      gram_tile_acc(acc, pa, X.x + (size_t)b * X.stride + 16 * h, X.Q);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int i = 32 * I + gram_acc_row(r, lane);
        if (i < cnt && jb < nb) {
          const float dt = DK == F32L2 ? (na[r] + nbn) - 2.0f * acc[r] : 1.0f - acc[r];
          const float eps = gram_eps<DK>(dt, na[r], nbn, A.d, false);
          const float up = dt + eps, lo = dt - eps;
          uint8_t c = UNSURE;
          if (up + fabsf(up) * u8 <= dva[r]) c = REJ;
          else if (lo - fabsf(lo) * u8 > dva[r]) c = KEEP;
          dec[i * 64 + jb] = c;
        }
      }
    }
  }
  wave_sync();
  // each candidate (lane) walks its row to the first rejection
  int j = 0;
  bool done = lane >= cnt, rej = false;
  while (true) {
    if (!done) {
      while (j < nb && dec[lane * 64 + j] == KEEP) j++;
      if (j == nb) done = true;
      else if (dec[lane * 64 + j] == REJ) done = rej = true;
    }
    const bool pend = !done;  // at an UNSURE test
    const uint64_t pm = ballot(pend);
    if (!pm) break;
    const int np = popc64(pm);
    if (pend) {
      const int q = popc64(pm & lanes_below());
      qv[q] = key_id(cdk[lane]);
      qb[q] = nbr[j];
    }
    wave_sync();
    for (int e0 = 0; e0 < np; e0 += G) {
      const int e = e0 + lane / L;
      const int ec = e < np ? e : 0;
      const float v = group_dist_stream<DK, L, NCH>(X.x + (size_t)qv[ec] * X.stride, X.x + (size_t)qb[ec] * X.stride,
                                                    X.Q, g);
      if (e < np && g == 0) qd[e] = v;
    }
    wave_sync();
    if (pend) {
      const float dvb = qd[popc64(pm & lanes_below())];
      if (dvb <= hi_to_float<DK>(key_hi(cdk[lane]))) done = rej = true;
      else j++;
    }
    wave_sync();
  }
  uint32_t tests = lane < cnt ? (uint32_t)(rej ? j + 1 : nb) : 0u;
  if (lane < cnt && rej) A.flag[sg.start + cpos[lane]] = 2;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) tests += __shfl_xor(tests, off, 64);
  *ev += tests;  // the same wave total in every lane, as the exact loop counts
  wave_sync();
}

// Reject every undecided candidate after the resolved chunk that one of the
// chunk's new neighbours occludes (d(v,b) <= d(v,a)), testing the new
// neighbours in acceptance order and stopping at the first that rejects.
template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_sat_filter(SatArgs A) {
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  __shared__ uint32_t cpos[64];
  __shared__ uint64_t cdk[64];
  __shared__ uint8_t dec[(DK != U8L2 && NCH >= 16) ? 64 * 64 : 1];
  const int lane = lane_id(), g = lane % L;
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  if (sg.nN == sg.nN_prev) return;
  const uint32_t lo = max(tl.off, sg.pos), hi = min(sg.len, tl.off + kTile);
  unsigned long long ev = 0;
  bool gram = false;
  if constexpr (DK != U8L2 && NCH >= 16) gram = A.norm != nullptr && sg.nN - sg.nN_prev <= 64;
  for (uint32_t base = lo; base < hi; base += 64) {
    uint32_t j = base + lane;
    bool und = j < hi && A.flag[sg.start + j] == 0;
    uint64_t m = ballot(und);
    if (!m) continue;
    if (und) {
      int r = popc64(m & lanes_below());
      cpos[r] = j;
      cdk[r] = A.key[sg.start + j];
    }
    wave_sync();
    int cnt = popc64(m);
    if constexpr (DK != U8L2 && NCH >= 16) {
      if (gram) {  // queue in cid and ckey (ids, then distances), decisions in dec
        filter_gram<DK, L, NCH>(A, sg, cnt, A.nl + sg.start + sg.nN_prev, (int)(sg.nN - sg.nN_prev), cpos, cdk,
                                dec, cid, reinterpret_cast<uint32_t*>(ckey), reinterpret_cast<float*>(ckey) + 64,
                                &ev);
        continue;
      }
    }
    for (uint32_t kb = sg.nN_prev; kb < sg.nN && cnt > 0; kb++) {
      uint32_t b = A.nl[sg.start + kb];
      Chunks<L, NCH> bc;
      const RowSet X = sat_rows<NCH>(A, sg.center);
      load_chunks<L, NCH>(bc, X.x + (size_t)b * X.stride, X.Q, g);
      uint32_t bn = 0;
      if constexpr (DK == U8L2) bn = group_sum_u32<L>(u8_selfdot<L, NCH>(bc));
      if (lane < cnt) cid[lane] = key_id(cdk[lane]);
      wave_sync();
      batch_dists_rs<DK, L, NCH>(X, bc, bn, cid, cnt, ckey);
      ev += (unsigned long long)cnt;
      bool keep = false;
      uint32_t mypos = 0;
      uint64_t mydk = 0;
      if (lane < cnt) {
        float dvb = hi_to_float<DK>(key_hi(ckey[lane]));
        float dva = hi_to_float<DK>(key_hi(cdk[lane]));
        mypos = cpos[lane];
        mydk = cdk[lane];
        keep = !(dvb <= dva);
        if (!keep) A.flag[sg.start + mypos] = 2;
      }
      uint64_t km = ballot(keep);
      wave_sync();
      if (keep) {
        int r = popc64(km & lanes_below());
        cpos[r] = mypos;
        cdk[r] = mydk;
      }
      cnt = popc64(km);
      wave_sync();
    }
  }
  if (lane == 0 && ev) atomicAdd(&A.counters[1], ev);
}

// Closest neighbour of each rejected candidate: argmin over the bag's
// neighbour list of (d(v,b), b).  The candidates stay in registers while
// the neighbours stream past.
template <int DK, int L, int NCH>
__device__ void argmin_wave(const RowSet& X, const uint32_t* cand, int ncand, const uint32_t* nbr,
                            int nn, uint32_t* owner_out, unsigned long long* ev) {
  constexpr int G = 64 / L;
  constexpr int RB = (NCH >= 8) ? 1 : ((8 / NCH) < L ? (8 / NCH) : L);
  const int lane = lane_id(), grp = lane / L, g = lane % L;
  for (int r0 = 0; r0 < ncand; r0 += G * RB) {
    Chunks<L, NCH> vc[RB];
    uint32_t vn[RB];
    uint64_t best[RB];
    uint32_t bidx[RB];
#pragma unroll
    for (int t = 0; t < RB; t++) {
      int r = r0 + t * G + grp;
      uint32_t v = cand[r < ncand ? r : 0];
      load_chunks<L, NCH>(vc[t], X.x + (size_t)v * X.stride, X.Q, g);
      vn[t] = 0;
      if constexpr (DK == U8L2) vn[t] = group_sum_u32<L>(u8_selfdot<L, NCH>(vc[t]));
      best[t] = FG_KEY_NONE;
      bidx[t] = 0;
    }
    for (int kb = 0; kb < nn; kb++) {
      uint32_t b = nbr[kb];
      Chunks<L, NCH> bc;
      load_chunks<L, NCH>(bc, X.x + (size_t)b * X.stride, X.Q, g);
#pragma unroll
      for (int t = 0; t < RB; t++) {
        uint32_t hi = group_dist<DK, L, NCH>(vc[t], vn[t], bc, X.Q, g);
        uint64_t kk = make_key(hi, b);
        if (kk < best[t]) {
          best[t] = kk;
          bidx[t] = (uint32_t)kb;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RB; t++) {
      int r = r0 + t * G + grp;
      if (r < ncand && g == 0) owner_out[r] = bidx[t];
    }
    int done = min(ncand - r0, G * RB);
    *ev += (unsigned long long)done * nn;
  }
  wave_sync();
}

// argmin_wave for float32 rows of more than 64 chunks, from 32x32 tiles of
// <v, b> on the matrix cores: d~(v,b) = |v|^2 + |b|^2 - 2<v,b> (cosine
// 1 - <v,b>) with the Gram-tile prune's margin eps.  Scanning the neighbours
// in 32-column blocks, each row keeps U = the least fl(d~ + eps) so far (an
// upper bound on its exact minimum); a pair whose fl(d~ - eps) is at most U
// might be the minimum and is queued.  U only falls, so every pair within
// the final bound is queued.  Queued pairs get the exact declared-order
// distance and the least key (distance, neighbour id) wins, as in
// argmin_wave.  LDS: best[64], qi[64], qj[64].
template <int DK, int L, int NCH>
__device__ void argmin_gram(const RowSet& X, int d, const float* norm, const uint32_t* cand, int ncand,
                            const uint32_t* nbr, int nn, uint32_t* owner_out, unsigned long long* ev,
                            uint64_t* best, uint32_t* qi, uint32_t* qj) {
  constexpr int G = 64 / L;
  const int lane = lane_id(), h = lane >> 5, g = lane % L;
  const float u8 = 8.0f * 5.9604645e-08f;
  best[lane] = FG_KEY_NONE;
  wave_sync();
  int qn = 0;
  auto flush = [&]() {
    for (int e0 = 0; e0 < qn; e0 += G) {
      const int e = e0 + lane / L;
      const int ec = e < qn ? e : 0;
      const uint32_t v = cand[qi[ec]], b = nbr[qj[ec]];
      const float dist = group_dist_stream<DK, L, NCH>(X.x + (size_t)v * X.stride, X.x + (size_t)b * X.stride,
                                                        X.Q, g);
      if (e < qn && g == 0) atomicMin(reinterpret_cast<unsigned long long*>(&best[qi[e]]),
                                      (unsigned long long)make_key(f32_to_ord(dist), b));
    }
    wave_sync();
    for (int e = lane; e < qn; e += 64)
      if (key_id(best[qi[e]]) == nbr[qj[e]]) owner_out[qi[e]] = qj[e];
    wave_sync();
    qn = 0;
  };
  for (int I = 0; 32 * I < ncand; I++) {
    const int ra = 32 * I + (lane & 31);
    const uint8_t* pa = X.x + (size_t)cand[ra < ncand ? ra : 0] * X.stride + 16 * h;
    float na[16], U[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int i = 32 * I + gram_acc_row(r, lane);
      na[r] = norm[cand[i < ncand ? i : 0]];
      U[r] = __builtin_inff();
    }
    for (int J = 0; 32 * J < nn; J++) {
      const int jb = 32 * J + (lane & 31);
      const uint32_t b = nbr[jb < nn ? jb : 0];
      const float nb = norm[b];
      gram_f32x16 acc;
#pragma unroll
      for (int e = 0; e < 16; e++) acc[e] = 0.0f;
      gram_tile_acc(acc, pa, X.x + (size_t)b * X.stride + 16 * h, X.Q);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int i = 32 * I + gram_acc_row(r, lane);
        const bool ok = jb < nn && i < ncand;
        const float dt = DK == F32L2 ? (na[r] + nb) - 2.0f * acc[r] : 1.0f - acc[r];
        const float eps = gram_eps<DK>(dt, na[r], nb, d, false);
        const float up = dt + eps, lo = dt - eps;
        float m = ok ? up + fabsf(up) * u8 : __builtin_inff();
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) m = fminf(m, __shfl_xor(m, off, 64));
        U[r] = fminf(U[r], m);
        const bool maybe = ok && lo - fabsf(lo) * u8 <= U[r];
        const uint64_t mq = ballot(maybe);
        const int nq = popc64(mq);
        if (nq == 0) continue;
        if (qn + nq > 64) flush();
        if (maybe) {
          const int pos = qn + popc64(mq & lanes_below());
          qi[pos] = (uint32_t)i;
          qj[pos] = (uint32_t)jb;
        }
        qn += nq;
        wave_sync();
      }
    }
  }
  if (qn) flush();
  *ev += (unsigned long long)ncand * nn;
}

template <int DK, int L, int NCH>
__global__ void __launch_bounds__(64) k_sat_assign(SatArgs A) {
  __shared__ uint32_t cand[64];
  __shared__ uint32_t cpos[64];
  __shared__ uint32_t own[64];
  __shared__ uint64_t gbest[64];
  __shared__ uint32_t gqi[64], gqj[64];
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kTile);
  unsigned long long ev = 0;
  for (uint32_t base = tl.off; base < hi; base += 64) {
    uint32_t j = base + lane;
    bool rej = j < hi && A.flag[sg.start + j] == 2;
    uint64_t m = ballot(rej);
    if (!m) continue;
    if (rej) {
      int r = popc64(m & lanes_below());
      cand[r] = A.perm[sg.start + j];
      cpos[r] = j;
    }
    wave_sync();
    int cnt = popc64(m);
    bool gram = false;
    if constexpr (DK != U8L2 && NCH >= 16) gram = A.norm != nullptr;
    if (gram)
      argmin_gram<DK, L, NCH>(A.X, A.d, A.norm, cand, cnt, A.nl + sg.start, (int)sg.nN, own, &ev, gbest, gqi, gqj);
    else
      argmin_wave<DK, L, NCH>(sat_rows<NCH>(A, sg.center), cand, cnt, A.nl + sg.start, (int)sg.nN, own, &ev);
    if (lane < cnt) A.owner[sg.start + cpos[lane]] = own[lane];
    wave_sync();
  }
  if (lane == 0 && ev) atomicAdd(&A.counters[2], ev);
}

// Count the members of each child bag.
// Bags with at most kBinMax children count (and, in k_sat_scatter, rank)
// their rejected points per child in LDS first, so a tile adds to each
// child's global counter once; the top levels have few children and would
// otherwise serialise millions of atomics on a handful of counters.
constexpr int kBinMax = 1024;

__global__ void __launch_bounds__(64) k_sat_count(SatArgs A) {
  __shared__ uint32_t bins[kBinMax];
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kTile);
  if (sg.nN > (uint32_t)kBinMax) {
    for (uint32_t j = tl.off + lane; j < hi; j += 64)
      if (A.flag[sg.start + j] == 2) atomicAdd(&A.ccount[sg.start + A.owner[sg.start + j]], 1u);
    return;
  }
  for (uint32_t k = lane; k < sg.nN; k += 64) bins[k] = 0;
  wave_sync();
  for (uint32_t j = tl.off + lane; j < hi; j += 64)
    if (A.flag[sg.start + j] == 2) atomicAdd(&bins[A.owner[sg.start + j]], 1u);
  wave_sync();
  for (uint32_t k = lane; k < sg.nN; k += 64)
    if (bins[k]) atomicAdd(&A.ccount[sg.start + k], bins[k]);
}
__global__ void __launch_bounds__(64) k_sat_children(SatArgs A) {
  const int lane = lane_id();
  const SatSeg sg = A.segs[blockIdx.x];
  uint32_t run = 0;
  for (uint32_t base = 0; base < sg.nN; base += 64) {
    uint32_t k = base + lane;
    uint32_t c = k < sg.nN ? A.ccount[sg.start + k] : 0;
    uint32_t inc = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t o = __shfl_up(inc, off, 64);
      if (lane >= off) inc += o;
    }
    uint32_t excl = run + inc - c;
    if (k < sg.nN) {
      uint32_t b = A.nl[sg.start + k];
      A.parent[(uint64_t)sg.t * A.n + b] = sg.center;
      A.perm2[sg.start + k] = b;
      A.coff[sg.start + k] = excl;
      A.ccount[sg.start + k] = 0;  // becomes the scatter cursor
      if (c > 0) {
        SatSeg ns;
        ns.t = sg.t;
        ns.center = b;
        ns.start = sg.start + sg.nN + excl;
        ns.len = c;
        ns.pos = 0;
        ns.nN = 0;
        ns.nN_prev = 0;
        if (c > (uint32_t)kSmall) {
          uint32_t at = atomicAdd(A.n_next, 1u);
          if (at < A.cap_next) A.next[at] = ns;
          else atomicOr(A.status, 8);
        } else {
          uint32_t at = atomicAdd(A.n_small, 1u);
          if (at < A.cap_small) A.small[at] = ns;
          else atomicOr(A.status, 8);
        }
      }
    }
    run += __shfl(inc, 63, 64);
  }
}

__global__ void __launch_bounds__(64) k_sat_scatter(SatArgs A) {
  __shared__ uint32_t bins[kBinMax];
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kTile);
  if (sg.nN > (uint32_t)kBinMax) {
    for (uint32_t j = tl.off + lane; j < hi; j += 64) {
      if (A.flag[sg.start + j] != 2) continue;
      uint32_t k = A.owner[sg.start + j];
      uint32_t at = atomicAdd(&A.ccount[sg.start + k], 1u);
      A.perm2[sg.start + sg.nN + A.coff[sg.start + k] + at] = A.perm[sg.start + j];
    }
    return;
  }
  // a bag's order does not matter: the next level sorts it by (distance, id)
  constexpr int kPer = kTile / 64;
  uint32_t rank[kPer], own[kPer];
  for (uint32_t k = lane; k < sg.nN; k += 64) bins[k] = 0;
  wave_sync();
#pragma unroll
  for (int it = 0; it < kPer; it++) {
    const uint32_t j = tl.off + it * 64 + lane;
    own[it] = FG_NONE;
    if (j < hi && A.flag[sg.start + j] == 2) {
      own[it] = A.owner[sg.start + j];
      rank[it] = atomicAdd(&bins[own[it]], 1u);
    }
  }
  wave_sync();
  for (uint32_t k = lane; k < sg.nN; k += 64)
    if (bins[k]) bins[k] = atomicAdd(&A.ccount[sg.start + k], bins[k]);
  wave_sync();
#pragma unroll
  for (int it = 0; it < kPer; it++) {
    const uint32_t j = tl.off + it * 64 + lane;
    if (own[it] != FG_NONE) {
      const uint32_t k = own[it];
      A.perm2[sg.start + sg.nN + A.coff[sg.start + k] + bins[k] + rank[it]] = A.perm[sg.start + j];
    }
  }
}
__global__ void __launch_bounds__(64) k_sat_copy_back(SatArgs A) {
  const int lane = lane_id();
  const SatTile tl = A.tiles[blockIdx.x];
  const SatSeg sg = A.segs[tl.seg];
  const uint32_t hi = min(sg.len, tl.off + kTile);
  for (uint32_t j = tl.off + lane; j < hi; j += 64) A.perm[sg.start + j] = A.perm2[sg.start + j];
}

// ---------------------------------------------------------------- small bags
// One wave builds the whole subtree of a small bag.  The stack lives in the
// bag's own range of the stack arrays (a subtree has at most len nodes).
constexpr int kSmallLo = 256;

template <int DK, int L, int NCH, int CAP>
__global__ void __launch_bounds__(64) k_sat_small(SatArgs A, uint32_t nsmall) {
  // bags of at most kSmallLo points take the instance with the small LDS
  // footprint (more waves per compute unit), larger ones the other
  constexpr bool kLo = CAP <= kSmallLo;
  __shared__ uint64_t sk[CAP];
  __shared__ uint32_t nb[CAP];
  __shared__ uint32_t own[CAP];
  __shared__ uint32_t cc[CAP];
  __shared__ uint32_t alive[CAP / 32];
  __shared__ uint32_t cid[64];
  __shared__ uint64_t ckey[64];
  const int lane = lane_id(), g = lane % L;
  unsigned long long ev_keys = 0, ev_acc = 0, ev_asg = 0;
  for (uint32_t si = blockIdx.x; si < nsmall; si += gridDim.x) {
    const SatSeg sg = A.small[si];
    if ((sg.len <= (uint32_t)kSmallLo) != kLo) continue;
    uint32_t* sa = A.stk_a + sg.start;
    uint32_t* ss = A.stk_s + sg.start;
    uint32_t* sm = A.stk_m + sg.start;
    int sp = 0;
    if (lane == 0) {
      sa[0] = sg.center;
      ss[0] = (uint32_t)sg.start;
      sm[0] = sg.len;
    }
    sp = 1;
    wave_sync();
    while (sp > 0) {
      sp--;
      const uint32_t a = sa[sp];
      const uint32_t s = ss[sp];
      const int m = (int)sm[sp];
      wave_sync();
      // keys (d(v, a), v)
      Chunks<L, NCH> ac;
      const RowSet X = sat_rows<NCH>(A, sg.center);
      load_chunks<L, NCH>(ac, X.x + (size_t)a * X.stride, X.Q, g);
      uint32_t an = 0;
      if constexpr (DK == U8L2) an = group_sum_u32<L>(u8_selfdot<L, NCH>(ac));
      for (int base = 0; base < m; base += 64) {
        int cnt = min(64, m - base);
        if (lane < cnt) cid[lane] = A.perm[s + base + lane];
        wave_sync();
        batch_dists_rs<DK, L, NCH>(X, ac, an, cid, cnt, sk + base);
      }
      ev_keys += (unsigned long long)m;
      int M = 64;
      while (M < m) M <<= 1;
      for (int i = m + lane; i < M; i += 64) sk[i] = FG_KEY_NONE;
      wave_sync();
      wave_sort_lds<uint64_t>(sk, M);
      // acceptance = prune with alpha 1, unbounded degree
      const int nn = prune_wave<DK, L, NCH>(X, 1.0f, m + 1, sk, m, alive, cid, ckey, nb, &ev_acc);
      wave_sync();
      // rejected candidates: closest neighbour
      int nrej = 0;
      for (int base = 0; base < M; base += 64) {
        int i = base + lane;
        bool rej = i < m && !((alive[i >> 5] >> (i & 31)) & 1u);
        uint64_t msk = ballot(rej);
        if (rej) cid[popc64(msk & lanes_below())] = key_id(sk[i]);
        wave_sync();
        int cnt = popc64(msk);
        if (cnt) {
          bool gram = false;
          if constexpr (DK != U8L2 && NCH >= 16) gram = A.norm != nullptr;
          if (gram)  // best in ckey, the queue in cc (free until the counts below)
            argmin_gram<DK, L, NCH>(A.X, A.d, A.norm, cid, cnt, nb, nn, own + nrej, &ev_asg, ckey, cc, cc + 64);
          else
            argmin_wave<DK, L, NCH>(X, cid, cnt, nb, nn, own + nrej, &ev_asg);
          if (lane < cnt) A.stk_tmp[s + nrej + lane] = cid[lane];  // id of rejected #(nrej + lane)
          nrej += cnt;
        }
        wave_sync();
      }
      // counts per child, offsets
      for (int k = lane; k < nn; k += 64) cc[k] = 0;
      wave_sync();
      for (int r = lane; r < nrej; r += 64) atomicAdd(&cc[own[r]], 1u);
      wave_sync();
      uint32_t run = 0;
      for (int base = 0; base < nn; base += 64) {
        int k = base + lane;
        uint32_t c = k < nn ? cc[k] : 0;
        uint32_t inc = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          uint32_t o = __shfl_up(inc, off, 64);
          if (lane >= off) inc += o;
        }
        if (k < nn) cc[k] = run + inc - c;  // exclusive offset
        run += __shfl(inc, 63, 64);
      }
      wave_sync();
      // new layout of [s, s+m): neighbours, then bags in neighbour order
      for (int k = lane; k < nn; k += 64) {
        A.perm[s + k] = nb[k];
        A.parent[(uint64_t)sg.t * A.n + nb[k]] = a;
      }
      // children first (their offsets), pushed in neighbour order
      for (int k = lane; k < nn; k += 64) {
        uint32_t start_k = cc[k];
        uint32_t end_k = (k + 1 < nn) ? cc[k + 1] : (uint32_t)nrej;
        uint32_t len_k = end_k - start_k;
        own[nrej + k] = len_k;  // stash lengths after the owners
      }
      wave_sync();
      // scatter rejected candidates (stable by rank) into their bags
      for (int r = lane; r < nrej; r += 64) {
        uint32_t k = own[r];
        uint32_t at = atomicAdd(&cc[k], 1u);
        A.perm[s + nn + at] = A.stk_tmp[s + r];
      }
      wave_sync();
      // push children with non-empty bags
      int pushed = 0;
      for (int base = 0; base < nn; base += 64) {
        int k = base + lane;
        uint32_t len_k = k < nn ? own[nrej + k] : 0;
        bool push = len_k > 0;
        uint64_t pm = ballot(push);
        if (push) {
          int at = sp + pushed + popc64(pm & lanes_below());
          uint32_t endk = cc[k];  // after scatter, cc[k] = end offset of bag k
          sa[at] = nb[k];
          ss[at] = s + (uint32_t)nn + endk - len_k;
          sm[at] = len_k;
        }
        pushed += popc64(pm);
      }
      sp += pushed;
      wave_sync();
    }
  }
  if (lane == 0) {
    atomicAdd(&A.counters[0], ev_keys);
    atomicAdd(&A.counters[1], ev_acc);
    atomicAdd(&A.counters[2], ev_asg);
  }
}

// ---------------------------------------------------------------- S_0
__global__ void k_tree_degrees(int64_t total, int64_t n, const uint32_t* parent, uint32_t* deg) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t p = parent[i];
    if (p == FG_NONE) continue;
    atomicAdd(&deg[i % n], 1u);
    atomicAdd(&deg[p], 1u);
  }
}

__global__ void k_tree_edges(int64_t total, int64_t n, const uint32_t* parent, const uint64_t* off,
                             uint32_t* cursor, uint32_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t p = parent[i];
    if (p == FG_NONE) continue;
    uint32_t v = (uint32_t)(i % n);
    out[off[v] + atomicAdd(&cursor[v], 1u)] = p;
    out[off[p] + atomicAdd(&cursor[p], 1u)] = v;
  }
}

template <int DK, int L, int NCH>
struct SatKernels {
  static void* keys() { return (void*)&k_sat_keys<DK, L, NCH>; }
  static void* resolve() { return (void*)&k_sat_resolve<DK, L, NCH>; }
  static void* filter() { return (void*)&k_sat_filter<DK, L, NCH>; }
  static void* assign() { return (void*)&k_sat_assign<DK, L, NCH>; }
  static void* small_lo() { return (void*)&k_sat_small<DK, L, NCH, kSmallLo>; }
  static void* small() { return (void*)&k_sat_small<DK, L, NCH, kSmall>; }
};

struct KSet {
  void *keys, *resolve, *filter, *assign, *small_lo, *small;
};

template <int DK, int L, int NCH>
KSet kset() {
  using K = SatKernels<DK, L, NCH>;
  return KSet{K::keys(), K::resolve(), K::filter(), K::assign(), K::small_lo(), K::small()};
}

bool pick_kset(int dk, int Q, KSet* k) {
  if (dk == U8L2) {
    if (Q <= 8) return *k = kset<U8L2, 8, 1>(), true;
    if (Q <= 16) return *k = kset<U8L2, 16, 1>(), true;
    return false;
  }
#define FG_F32_ROWS(DKV)                                   \
  if (Q <= 8) return *k = kset<DKV, 8, 1>(), true;         \
  if (Q <= 16) return *k = kset<DKV, 16, 1>(), true;       \
  if (Q <= 32) return *k = kset<DKV, 16, 2>(), true;       \
  if (Q <= 64) return *k = kset<DKV, 16, 4>(), true;       \
  if (Q <= 256) return *k = kset<DKV, 16, 16>(), true;     \
  return false;
  if (dk == F32L2) { FG_F32_ROWS(F32L2) }
  if (dk == F32COS) { FG_F32_ROWS(F32COS) }
#undef FG_F32_ROWS
  return false;
}

hipError_t launch(void* k, unsigned grid, SatArgs& a, hipStream_t st) {
  if (grid == 0) return hipSuccess;
  void* args[] = {&a};
  return hipLaunchKernel(k, dim3(grid), dim3(64), args, 0, st);
}

int blocks_for(int64_t count, int per_block) {
  int64_t b = (count + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

}  // namespace

hipError_t sat_iota(uint32_t* perm, int64_t n, uint32_t T, int64_t off, int64_t ni, const uint32_t* roots,
                    hipStream_t st);
hipError_t sat_clear_counts(SatArgs& a, unsigned nt, hipStream_t st);

namespace {
// |x_i|^2 of every float32 row, one wave per row (four elements per lane
// step, then a wave sum).
__global__ void __launch_bounds__(256) k_sat_norms(const uint8_t* x, int64_t stride, int64_t n, int Q,
                                                   float* out) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    float s = 0.0f;
    for (int c = lane; c < Q; c += 64) {
      const float4 v = *reinterpret_cast<const float4*>(x + i * stride + 16 * (int64_t)c);
      s = __builtin_fmaf(v.x, v.x, s);
      s = __builtin_fmaf(v.y, v.y, s);
      s = __builtin_fmaf(v.z, v.z, s);
      s = __builtin_fmaf(v.w, v.w, s);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[i] = s;
  }
}
}  // namespace

hipError_t row_sq_norms(const Shape& s, float* out, hipStream_t st) {
  k_sat_norms<<<(unsigned)blocks_for(s.n, 4), 256, 0, st>>>(s.x, s.stride, s.n, s.Q, out);
  return hipGetLastError();
}

size_t sat_workspace_bytes(int64_t n, uint32_t T, SatWs* w) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const uint64_t tn = (uint64_t)T * n;
  w->perm = take(tn * 4);
  w->perm2 = take(tn * 4);
  w->key = take(tn * 8);
  w->key2 = take(tn * 8);
  w->flag = take(tn);
  w->owner = take(tn * 4);
  w->nl = take(tn * 4);
  w->ccount = take(tn * 4);
  w->coff = take(tn * 4);
  w->stk_a = take(tn * 4);
  w->stk_s = take(tn * 4);
  w->stk_m = take(tn * 4);
  w->stk_tmp = take(tn * 4);
  w->cap_segs = (uint32_t)(tn / kSmall + T + 64);
  w->segs = take((size_t)w->cap_segs * sizeof(SatSeg));
  w->next = take((size_t)w->cap_segs * sizeof(SatSeg));
  w->cap_small = (uint32_t)(tn / 2 + 64);
  w->small = take((size_t)w->cap_small * sizeof(SatSeg));
  w->cap_tiles = (uint32_t)(tn / kTile + 2 * w->cap_segs + 64);
  w->tiles = take((size_t)w->cap_tiles * sizeof(SatTile));
  w->ctl = take(4096);
  w->norm = take((uint64_t)n * 4);
  w->total = o;
  return o;
}

// Build the T trees.  parent (T x n, device) receives every tree's parent
// array; counters[0..2] (device) accumulate distance evaluations.
hipError_t sat_build(const Shape& s, const uint32_t* roots, uint32_t T, uint32_t* parent, char* ws,
                     const SatWs& w, hipStream_t st, unsigned long long* host_evals, int* host_status) {
  std::vector<uint32_t> hroots(T);
  hipError_t e = hipMemcpyAsync(hroots.data(), roots, T * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  std::vector<SatInstance> one{SatInstance{0, s.n, hroots.data()}};
  return sat_build_multi(s, T, one, parent, ws, w, st, host_evals, host_status);
}

hipError_t sat_build_multi(const Shape& s, uint32_t T, const std::vector<SatInstance>& inst, uint32_t* parent,
                           char* ws, const SatWs& w, hipStream_t st, unsigned long long* host_evals,
                           int* host_status, const uint16_t* inst_of, const int* inst_q) {
  KSet K;
  if (!pick_kset(s.dk, s.Q, &K)) return hipErrorInvalidValue;
  if (T > 64) return hipErrorInvalidValue;
  const int64_t n = s.n;
  SatArgs a{};
  a.X = RowSet{s.x, s.stride, s.Q};
  a.n = n;
  a.perm = reinterpret_cast<uint32_t*>(ws + w.perm);
  a.perm2 = reinterpret_cast<uint32_t*>(ws + w.perm2);
  a.key = reinterpret_cast<uint64_t*>(ws + w.key);
  a.flag = reinterpret_cast<uint8_t*>(ws + w.flag);
  a.owner = reinterpret_cast<uint32_t*>(ws + w.owner);
  a.nl = reinterpret_cast<uint32_t*>(ws + w.nl);
  a.ccount = reinterpret_cast<uint32_t*>(ws + w.ccount);
  a.coff = reinterpret_cast<uint32_t*>(ws + w.coff);
  a.stk_a = reinterpret_cast<uint32_t*>(ws + w.stk_a);
  a.stk_s = reinterpret_cast<uint32_t*>(ws + w.stk_s);
  a.stk_m = reinterpret_cast<uint32_t*>(ws + w.stk_m);
  a.stk_tmp = reinterpret_cast<uint32_t*>(ws + w.stk_tmp);
  a.parent = parent;
  a.segs = reinterpret_cast<SatSeg*>(ws + w.segs);
  a.next = reinterpret_cast<SatSeg*>(ws + w.next);
  a.cap_next = w.cap_segs;
  a.small = reinterpret_cast<SatSeg*>(ws + w.small);
  a.cap_small = w.cap_small;
  a.tiles = reinterpret_cast<SatTile*>(ws + w.tiles);
  SatCtl* ctl = reinterpret_cast<SatCtl*>(ws + w.ctl);
  a.counters = ctl->counters;
  a.active = &ctl->active;
  a.n_next = &ctl->n_next;
  a.n_small = &ctl->n_small;
  a.status = &ctl->status;
  a.d = s.d;
  a.inst_of = inst_of;
  a.inst_q = inst_of ? inst_q : nullptr;
  hipError_t e;
#define CK(x)                       \
  do {                              \
    e = (x);                        \
    if (e != hipSuccess) return e;  \
  } while (0)

  const uint64_t tn = (uint64_t)T * n;
  CK(fill_u32(reinterpret_cast<uint32_t*>(ctl), 0, sizeof(SatCtl) / 4, st));
  CK(fill_u32(parent, FG_NONE, (int64_t)tn, st));
  CK(fill_u32(a.ccount, 0, (int64_t)tn, st));
  if (s.dk != U8L2 && s.Q > 64 && s.d <= 1024) {  // the matrix-core assignment's norms
    float* nrm = reinterpret_cast<float*>(ws + w.norm);
    k_sat_norms<<<(unsigned)blocks_for(n, 4), 256, 0, st>>>(s.x, s.stride, n, s.Q, nrm);
    CK(hipGetLastError());
    a.norm = nrm;
  }
  // Tree t of instance i: its first bag at positions [t*n + off, t*n + off +
  // n_i - 1) holds every id of the instance but its root.
  std::vector<SatSeg> large, init_small;
  for (const SatInstance& in : inst) {
    if (in.n <= 1) continue;
    CK(sat_iota(a.perm, n, T, in.off, in.n, in.roots, st));
    for (uint32_t t = 0; t < T; t++) {
      SatSeg sg{};
      sg.t = t;
      sg.center = (uint32_t)(in.off + in.roots[t]);
      sg.start = (uint64_t)t * n + (uint64_t)in.off;
      sg.len = (uint32_t)(in.n - 1);
      (sg.len > (uint32_t)kSmall ? large : init_small).push_back(sg);
    }
  }
  if (init_small.size() > w.cap_small) return hipErrorOutOfMemory;
  uint32_t n_small_host = (uint32_t)init_small.size();
  if (n_small_host) {
    CK(hipMemcpyAsync(a.small, init_small.data(), init_small.size() * sizeof(SatSeg),
                      hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(&ctl->n_small, &n_small_host, 4, hipMemcpyHostToDevice, st));
  }

  std::vector<SatTile> tiles;
  while (!large.empty()) {
    const uint32_t nseg = (uint32_t)large.size();
    if (nseg > w.cap_segs) return hipErrorOutOfMemory;
    tiles.clear();
    uint32_t maxlen = 0;
    for (uint32_t i = 0; i < nseg; i++) {
      for (uint32_t off = 0; off < large[i].len; off += kTile) tiles.push_back(SatTile{i, off});
      maxlen = std::max(maxlen, large[i].len);
    }
    if (tiles.size() > w.cap_tiles) return hipErrorOutOfMemory;
    const unsigned nt = (unsigned)tiles.size();
    CK(hipMemcpyAsync(a.segs, large.data(), nseg * sizeof(SatSeg), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(a.tiles, tiles.data(), nt * sizeof(SatTile), hipMemcpyHostToDevice, st));
    // 1. keys and sort
    CK(launch(K.keys, nt, a, st));
    CK(launch((void*)&k_sat_tile_sort, nt, a, st));
    uint64_t* src = a.key;
    uint64_t* dst = reinterpret_cast<uint64_t*>(ws + w.key2);
    for (uint32_t wdt = kTile; wdt < maxlen; wdt *= 2) {
      void* args[] = {&a, &src, &dst, &wdt};
      CK(hipLaunchKernel((void*)&k_sat_merge_pass, dim3(nt), dim3(64), args, 0, st));
      std::swap(src, dst);
    }
    uint64_t* key_orig = a.key;
    a.key = src;  // sorted keys
    CK(launch((void*)&k_sat_perm_from_keys, nt, a, st));
    // 2. acceptance rounds, four per check on the host: a round changes
    // nothing on a bag whose candidates are all decided (resolve returns,
    // filter finds no new neighbours), so the rounds after the last useful
    // one are empty launches
    for (;;) {
      for (int r = 0; r < 4; r++) {
        CK(fill_u32(&ctl->active, 0, 1, st));
        CK(launch(K.resolve, nseg, a, st));
        CK(launch(K.filter, nt, a, st));
      }
      uint32_t active = 0;
      CK(hipMemcpyAsync(&active, &ctl->active, 4, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      if (!active) break;
    }
    // 3. assignment and partition
    CK(launch(K.assign, nt, a, st));
    CK(launch((void*)&k_sat_count, nt, a, st));
    CK(fill_u32(&ctl->n_next, 0, 1, st));
    CK(launch((void*)&k_sat_children, nseg, a, st));
    CK(launch((void*)&k_sat_scatter, nt, a, st));
    CK(launch((void*)&k_sat_copy_back, nt, a, st));
    // clear the used child counters for the next level
    CK(sat_clear_counts(a, nt, st));
    a.key = key_orig;
    // 4. next level
    uint32_t nn = 0;
    int status = 0;
    CK(hipMemcpyAsync(&nn, &ctl->n_next, 4, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&status, &ctl->status, 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (status) {
      *host_status = status;
      return hipSuccess;
    }
    large.resize(nn);
    if (nn) {
      CK(hipMemcpyAsync(large.data(), a.next, nn * sizeof(SatSeg), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
    }
  }
  // 5. small bags
  uint32_t nsmall = 0;
  CK(hipMemcpyAsync(&nsmall, &ctl->n_small, 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (nsmall) {
    unsigned grid = nsmall < 65536 ? nsmall : 65536;
    void* args[] = {&a, &nsmall};
    CK(hipLaunchKernel(K.small_lo, dim3(grid), dim3(64), args, 0, st));
    CK(hipLaunchKernel(K.small, dim3(grid), dim3(64), args, 0, st));
  }
  unsigned long long ev[3];
  int status = 0;
  CK(hipMemcpyAsync(ev, ctl->counters, sizeof(ev), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(&status, &ctl->status, 4, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  *host_evals = ev[0] + ev[1] + ev[2];
  *host_status = status;
  return hipSuccess;
#undef CK
}

namespace {
struct RootList {
  uint32_t r[64];
};
// Tree t's first bag of one instance (ids [off, off + ni)): every id but
// off + root_t, in id order.
__global__ void k_sat_iota(uint32_t* perm, int64_t n, uint32_t T, int64_t off, int64_t ni, RootList roots) {
  int64_t total = (int64_t)T * (ni - 1);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = i / (ni - 1), j = i - t * (ni - 1);
    uint32_t r = roots.r[t];
    perm[t * n + off + j] = (uint32_t)(off + (j < (int64_t)r ? j : j + 1));
  }
}
__global__ void __launch_bounds__(64) k_sat_clear_counts(SatArgs A) {
  const SatSeg sg = A.segs[A.tiles[blockIdx.x].seg];
  const SatTile tl = A.tiles[blockIdx.x];
  const uint32_t hi = min(sg.nN, tl.off + kTile);
  for (uint32_t j = tl.off + lane_id(); j < hi; j += 64) A.ccount[sg.start + j] = 0;
}
}  // namespace

hipError_t sat_iota(uint32_t* perm, int64_t n, uint32_t T, int64_t off, int64_t ni, const uint32_t* roots,
                    hipStream_t st) {
  if (ni <= 1) return hipSuccess;
  RootList rl{};
  for (uint32_t t = 0; t < T && t < 64; t++) rl.r[t] = roots[t];
  k_sat_iota<<<blocks_for((int64_t)T * (ni - 1), 256), 256, 0, st>>>(perm, n, T, off, ni, rl);
  return hipGetLastError();
}

hipError_t sat_clear_counts(SatArgs& a, unsigned nt, hipStream_t st) {
  return launch((void*)&k_sat_clear_counts, nt, a, st);
}

hipError_t tree_edges_csr(int64_t n, uint32_t T, const uint32_t* parent, uint32_t* deg,
                          uint64_t* off_tmp, uint32_t* cursor, uint32_t* tmp_ids, hipStream_t st,
                          void* scan_scratch) {
  const int64_t total = (int64_t)T * n;
  hipError_t e = fill_u32(deg, 0, n, st);
  if (e != hipSuccess) return e;
  k_tree_degrees<<<blocks_for(total, 256), 256, 0, st>>>(total, n, parent, deg);
  e = exclusive_scan_u32_u64(deg, off_tmp, n, scan_scratch, st);
  if (e != hipSuccess) return e;
  e = fill_u32(cursor, 0, n, st);
  if (e != hipSuccess) return e;
  k_tree_edges<<<blocks_for(total, 256), 256, 0, st>>>(total, n, parent, off_tmp, cursor, tmp_ids);
  return hipGetLastError();
}

}  // namespace fg
