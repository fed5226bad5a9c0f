// The small-query size class: a range [a, b) of at most T integers (one LDS
// tile) handled from start to end by one workgroup, with no entry written to
// HBM and no partition or join launch.  The workgroup sieves rad(x) for x in
// [a, b] (Algorithm 1 on one tile: the dense prime powers from the static
// schedule of the T-value tile, every other power q <= b at its one possible
// multiple), applies the member test, takes the fingerprint of every kept set
// {rad(x), rad(x+1)} (of the query too, in batched calls) and joins them in an
// LDS hash table as the partition join does (Algorithm 3's insert step: every
// earlier equal fingerprint on the probe chain is a candidate).  Candidates go
// to the same verification as those of the passes.
#pragma once
#include "bx_kernels.h"

namespace bx {

struct SmallParams {
  const Query* queries;
  const uint32_t* list;  // indices of the small queries, one per workgroup
  int batch;
  uint32_t prune;
  const PrimePow* pp;
  uint32_t n_pp, n_dense;  // pp[0, n_dense) are the powers of the dense schedule (q <= T)
  const DenseTab* dense;
  uint64_t fp_mask;
  Cand* cand;
  uint32_t cand_cap;
  uint32_t* flags;
  unsigned long long* acc;  // acc[kAccEntries], acc[kAccJoined]
};

// T: the largest query length served (2048 or 8192, the tiles with a dense
// schedule); BLOCK threads per workgroup.
template <int T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_small(SmallParams P) {
  constexpr int ITER = T / BLOCK;
  constexpr int SLOTS = (dense_slot_cap(T) + BLOCK - 1) / BLOCK;
  constexpr uint32_t kSlots = 2 * T;  // load <= 0.5
  constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  constexpr uint32_t kIdxMask = (1u << kJoinIdxBits) - 1;
  static_assert(T % BLOCK == 0 && T < (1 << kJoinIdxBits), "tile and index field");
  __shared__ uint64_t tile[T + 1];  // rad(a + i); then the fingerprint of each kept i
  __shared__ uint32_t table[kSlots];
  __shared__ uint32_t doff[kDenseMax];
  __shared__ uint32_t n_act_s, kept_s;
  const int tid = threadIdx.x;
  const uint32_t qi = P.list[blockIdx.x];
  const uint64_t qa = P.queries[qi].a, qb = P.queries[qi].b;
  const uint32_t L = static_cast<uint32_t>(qb - qa);  // 2 <= L <= T (checked by the host)
  const uint32_t grp = P.batch ? qi : 0u;
  const DenseTab* D = P.dense;
  // Start values: a + i with the factor 2 reduced, for i in [0, L].
  for (uint32_t i = tid; i <= L; i += BLOCK) tile[i] = strip_two(qa + i);
  if (static_cast<uint32_t>(tid) < D->n) {
    const uint32_t q = D->q[tid];
    const uint32_t r = static_cast<uint32_t>(qa % q);
    doff[tid] = r ? q - r : 0u;
  }
  if (tid == 0) {
    // Powers up to b: pp is ascending.
    uint32_t l = P.n_dense, h = P.n_pp;
    while (l < h) {
      const uint32_t m = (l + h) >> 1;
      if (P.pp[m].q <= qb)
        l = m + 1;
      else
        h = m;
    }
    n_act_s = l;
    kept_s = 0;
  }
  __syncthreads();
  // Dense powers: this thread's slots of the static schedule.
#pragma unroll
  for (int k = 0; k < SLOTS; ++k) {
    const uint32_t t = tid + k * BLOCK;
    if (t < D->nslots) {
      const uint32_t d = D->slot_d[t];
      const uint32_t pos = doff[d] + (t - D->prefix[d]) * D->q[d];
      if (pos <= L) lds_div(&tile[pos], D->p[d], D->pinv[d]);
    }
  }
  // The other powers (q > T >= L) have at most one multiple in [a, b].
  const uint32_t n_act = n_act_s;
  for (uint32_t idx = P.n_dense + tid; idx < n_act; idx += BLOCK) {
    const PrimePow pw = P.pp[idx];
    const uint64_t r = mod_fp64(qa, pw.q, pw.invq);
    if (r == 0 || pw.q - r <= L) lds_div(&tile[r ? pw.q - r : 0], pw.p, pw.pinv);
  }
  __syncthreads();
  // Member test and fingerprints (kept in registers until every thread has
  // read its radicals, then written over them).
  uint64_t fp[ITER];
  uint32_t mine = 0;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t i = it * BLOCK + tid;
    fp[it] = ~0ull;
    if (i < L) {
      const uint64_t r0 = tile[i], r1 = tile[i + 1];
      if (!P.prune || may_pair(qa + i, r0, r1, qb)) {
        const uint64_t h = key64(r0 < r1 ? r0 : r1, r0 < r1 ? r1 : r0, grp);
        fp[it] = (h >> 11) & P.fp_mask;
        ++mine;
      }
    }
  }
  for (uint32_t s = tid; s < kSlots; s += BLOCK) table[s] = kEmpty;
  if (mine) atomicAdd(&kept_s, mine);
  __syncthreads();
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const uint32_t i = it * BLOCK + tid;
    if (i < L) tile[i] = fp[it];
  }
  __syncthreads();
  if (tid == 0 && kept_s) {
    atomicAdd(&P.acc[kAccEntries], static_cast<unsigned long long>(kept_s));
    atomicAdd(&P.acc[kAccJoined], static_cast<unsigned long long>(kept_s));
  }
  // Inserts: each walks its probe chain to the first empty slot and compares
  // with every occupied slot whose tag matches.  Equal fingerprints walk the
  // same chain, so the one that claims the later slot reports the pair (once).
  const uint64_t qbits = static_cast<uint64_t>(qi) << kGrpShift;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    if (fp[it] == ~0ull) continue;
    const uint32_t i = it * BLOCK + tid;
    const uint32_t h = static_cast<uint32_t>(fp[it]);
    const uint32_t word = (h & ~kIdxMask) | i;
    uint32_t s = h & (kSlots - 1);
    for (;;) {
      const uint32_t v = atomicCAS(&table[s], kEmpty, word);
      if (v == kEmpty) break;
      const uint32_t o = v & kIdxMask;
      if (((v ^ word) & ~kIdxMask) == 0 && tile[o] == fp[it]) {
        const uint32_t k = atomicAdd(&P.flags[kFlagCand], 1u);
        if (k < P.cand_cap) {
          Cand c;
          c.a = make_entry(P.batch ? (i | qbits) : qa + i, fp[it]);
          c.b = make_entry(P.batch ? (o | qbits) : qa + o, fp[it]);
          P.cand[k] = c;
        }
      }
      s = (s + 1) & (kSlots - 1);
    }
  }
}

}  // namespace bx
