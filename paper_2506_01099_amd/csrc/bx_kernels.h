// HIP kernels of the Benelux-pair search for gfx950.
//
//   k_sieve<MODE_RAD>   Algorithm 1 on LDS tiles, radicals written to HBM.
//   k_sieve<MODE_KEYS>  Algorithm 1 on LDS tiles, then for every x the member
//                       test (may_pair), the pass filter of the hash-
//                       partitioned passes, a fingerprint of the set S_x
//                       (Section 2.1), wave-ballot compaction and the first
//                       partition scatter of the join, fused in one kernel.
//   k_partition         second partition scatter (fan-out B2), XCD-aware.
//   k_join              LDS hash join of one partition: inserts that detect
//                       every earlier equal fingerprint on their probe chain,
//                       as the insert step of Algorithm 3 does, so each pair
//                       of a group of equal sets is reported exactly once.
//   k_verify            every candidate pair recomputed by trial division with
//                       the resident primes (equal fingerprints of different
//                       sets are dropped here), classified (first kind when
//                       rad(m) = rad(n), Algorithm 2) and filtered by kind.
//   k_fill_u32          fills a word array (clears counters inside graphs).
//   k_set_query         writes a one-query table from kernel arguments.
#pragma once
#include <type_traits>

#include "bx_device.h"

namespace bx {

constexpr int MODE_RAD = 0;
constexpr int MODE_KEYS = 1;

// Sparse-hit list held in LDS per segment (about 850 hits per 2^18 values
// with the 8192 tile, 2050 with the 2048 tile); the excess goes to a global
// spill list.
template <int T>
constexpr int hit_cap() { return 1024; }
constexpr int kB1Max = 1024;       // first partition fan-out
constexpr int kB2Max = 2048;       // second partition fan-out
constexpr int kPartChunk = 8192;   // entries per workgroup in k_partition
constexpr uint32_t kKindThird = 4; // kinds bit: also test rad(m + 2) = rad(n + 2)
constexpr int kJoinCap = 8192;     // entries of one LDS join chunk (held in registers)
constexpr int kJoinSlots = 16384;  // LDS hash-table slots (load <= 0.5)
constexpr int kJoinIdxBits = 14;   // slot = tag (18 bits) << 14 | entry index

struct SieveParams {
  const Query* queries;
  const uint64_t* seg_prefix;  // n_queries + 1: first segment of each query
  uint32_t n_queries;
  uint64_t n_segs;
  uint32_t seg_len;
  const PrimePow* pp;  // all odd prime powers <= hi_max, ascending
  uint32_t n_pp;
  uint32_t n_dense;  // pp[0, n_dense) are the dense ones (q <= tile)
  const DenseTab* dense;
  uint64_t* spill;  // per workgroup: spill + blockIdx.x * spill_cap
  uint32_t spill_cap;
  uint32_t* flags;
  // MODE_RAD
  uint64_t* rad_out;
  uint64_t rad_lo, rad_hi;
  // MODE_KEYS
  int batch;
  uint32_t prune;         // drop x that cannot be a member of any pair (may_pair)
  uint32_t pfilter;       // keep x only when pass_hash(key) is in [ph_lo, ph_hi)
  uint64_t ph_lo, ph_hi;
  uint32_t b1mask;  // first-level bucket = low bits of key64
  Entry* l1;       // region (b, w) of bucket b written by workgroup w: l1 + (b * gridDim.x + w) * cap1
  uint64_t cap1;   // entries per region
  uint32_t* cnt1;  // B1 x gridDim.x fill counts, written at the end of the kernel
};

template <int T, int BLOCK>
struct SieveShCommon {
  uint64_t tile[T + 1];
  uint64_t hits[hit_cap<T>()];
  uint32_t dres[kDenseMax], doff[kDenseMax], dq[kDenseMax], dtq[kDenseMax];
  uint32_t hit_n, n_act, stage_n, pad0;
  uint32_t wsum[BLOCK / 64];
};

// The stage collects the kept entries of several tiles; it is written out when
// less than kMargin slots are free at the start of a tile.  A flush runs
// between tiles, when the tile array is free: its counting sort keeps its
// histogram, offsets and permutation there (FlushScratch).
template <int T, int BLOCK>
struct SieveShKeys : SieveShCommon<T, BLOCK> {
  // Stage capacity: 6016 entries with the 8192 tile (one workgroup per CU:
  // what the LDS leaves beside the 64 KB tile), one tile with the 2048 tile
  // (two per CU).  The margin holds what a tile keeps in the bulk of a range
  // (0.107 T on average, below 0.125 T); a tile that keeps more sends the
  // excess straight to HBM.
  static constexpr int kStage = T >= 8192 ? 6016 : T;
  static constexpr int kMargin = T >= 8192 ? 1152 : T / 4;
  Entry stage[kStage];
  uint16_t sb[kStage];
  uint32_t lcur[kB1Max];
  struct FlushScratch {
    uint32_t cnt[kB1Max], gofs[kB1Max];
    uint16_t perm[kStage];
  };
  static_assert(sizeof(FlushScratch) <= sizeof(uint64_t) * (T + 1), "flush scratch must fit in the tile");
  __device__ FlushScratch* flush_scratch() { return reinterpret_cast<FlushScratch*>(this->tile); }
};

template <int T, int BLOCK, int MODE>
struct SieveShSel {
  using type = SieveShCommon<T, BLOCK>;
};
template <int T, int BLOCK>
struct SieveShSel<T, BLOCK, MODE_KEYS> {
  using type = SieveShKeys<T, BLOCK>;
};

// Counting sort of n staged entries (bucket of entry i in sb[i]) into runs per
// bucket: LDS histogram, one global reservation per non-empty bucket, then the
// runs are written with consecutive threads on consecutive entries (coalesced
// stores).  cnt/gofs hold NB words; perm holds n.  gcur[b] is the cursor of
// bucket b: shared by all workgroups (global, one atomic per non-empty bucket)
// or, with PRIVATE, owned by this workgroup (no atomics).  dst(b, k) stores the
// k-th entry of the bucket (k < cap).
template <int BLOCK, int NB, int NMAX, bool PRIVATE, typename Item, typename Bucket, typename Dst, typename Mid>
__device__ void scatter_runs(uint32_t n, uint32_t nb, const Item* ent, Bucket sb, uint16_t* perm,
                             uint32_t* cnt, uint32_t* gofs, uint32_t* wsum, uint32_t* gcur, uint64_t cap,
                             uint32_t* flag, Dst dst, Mid mid) {
  constexpr int BINS = (NB + BLOCK - 1) / BLOCK;
  // n <= NMAX: each thread takes the U entries tid + u * BLOCK, and every
  // step issues the LDS reads and atomics of all of them before it waits on
  // any (a thread past n reads entry 0 and leaves it alone).
  constexpr int U = (NMAX + BLOCK - 1) / BLOCK;
  const int tid = threadIdx.x;
  for (uint32_t b = tid; b < nb; b += BLOCK) cnt[b] = 0;
  __syncthreads();
  uint32_t bk[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t i = tid + u * BLOCK;
    bk[u] = sb(i < n ? i : 0u);
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (tid + u * BLOCK < n) atomicAdd(&cnt[bk[u]], 1u);
  __syncthreads();
  uint32_t loc[BINS];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < BINS; ++k) {
    const uint32_t b = tid * BINS + k;
    loc[k] = b < nb ? cnt[b] : 0u;
    sum += loc[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan<BLOCK>(sum, wsum, &tot);
#pragma unroll
  for (int k = 0; k < BINS; ++k) {
    const uint32_t b = tid * BINS + k;
    if (b < nb) {
      uint32_t g;
      if constexpr (PRIVATE) {  // gcur is this workgroup's own cursor array (LDS)
        g = gcur[b];
        gcur[b] = g + loc[k];
      } else {
        g = loc[k] ? atomicAdd(&gcur[b], loc[k]) : 0u;
      }
      gofs[b] = g - ex;  // slot j of the sorted order lands at run position g + (j - ex)
      cnt[b] = ex;       // becomes the LDS cursor of bucket b
    }
    ex += loc[k];
  }
  __syncthreads();
  mid();  // the global cursors are taken: work that may overlap the scatter
  uint32_t slot[U];
#pragma unroll
  for (int u = 0; u < U; ++u)
    slot[u] = tid + u * BLOCK < n ? atomicAdd(&cnt[bk[u]], 1u) : 0u;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (tid + u * BLOCK < n) perm[slot[u]] = static_cast<uint16_t>(tid + u * BLOCK);
  __syncthreads();
  uint32_t pi[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t j = tid + u * BLOCK;
    pi[u] = perm[j < n ? j : 0u];
  }
  uint32_t pb[U];
  Item pe[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    pb[u] = sb(pi[u]);
    pe[u] = ent[pi[u]];
  }
  uint32_t pk[U];
#pragma unroll
  for (int u = 0; u < U; ++u) pk[u] = gofs[pb[u]] + tid + u * BLOCK;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (tid + u * BLOCK < n) {
      if (pk[u] < cap)
        dst(pb[u], pk[u], pe[u]);
      else
        atomicOr(flag, 1u);
    }
  }
  __syncthreads();
}

// Entry of the kept integer x = x0 + i with rad(x) = a and rad(x + 1) = b;
// *bucket receives its first-level bucket.
__device__ __forceinline__ Entry kept_entry(const SieveParams& P, uint64_t a, uint64_t b, uint64_t x, uint64_t qa,
                                            uint32_t grp, uint32_t* bucket) {
  const uint64_t klo = a < b ? a : b, khi = a < b ? b : a;
  const uint64_t h = key64(klo, khi, grp);
  const uint64_t pos43 = P.batch ? ((x - qa) | (static_cast<uint64_t>(grp) << kGrpShift)) : x;
  *bucket = static_cast<uint32_t>(h) & P.b1mask;
  return make_entry(pos43, h >> 11);
}

// Orders the LDS accesses of one wave (its lanes share stage slots).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane mask of the wave's integers x (one per lane, rad(x) = r0 and
// rad(x + 1) = r1) that pass the member test (may_pair) for the query end qb.
// UPPER: the tile lies above qb / 2, where no squarefree x or x + 1 passes
// (the factor t is at least 2), so only both-non-squarefree x remain.  Below,
// a squarefree y of {x, x + 1} needs y * M <= qb with M = max(2, rad(other)
// - 1); M > lim_hi fails for the whole segment and settles almost every such
// y at once, M <= lim_lo passes for the whole segment, and the rare rest take
// the exact product.  small: the tile starts at x0 <= 3, where x <= 3 is kept.
template <bool UPPER>
__device__ __forceinline__ uint64_t member_mask(uint64_t x, uint64_t r0, uint64_t r1, uint64_t lim_hi, uint64_t lim_lo,
                                                uint64_t qb, bool small) {
  const bool s0 = r0 == x, s1 = r1 == x + 1;  // x, x + 1 squarefree
  uint64_t km = ~(__ballot(s0) | __ballot(s1));
  if constexpr (!UPPER) {
    const bool c0 = s0 && r1 <= lim_hi + 1, c1 = s1 && r0 <= lim_hi + 1;
    const uint64_t cm = __ballot(c0 || c1);
    if (cm) {
      bool k = false;
      if (c0 || c1) {
        const uint64_t M0 = r1 >= 3 ? r1 - 1 : 2, M1 = r0 >= 3 ? r0 - 1 : 2;
        const bool p0 = !s0 || (c0 && (M0 <= lim_lo || prod_le(x, M0, qb)));
        const bool p1 = !s1 || (c1 && (M1 <= lim_lo || prod_le(x + 1, M1, qb)));
        k = p0 && p1;
      }
      km = (km & ~cm) | __ballot(k);
    }
    if (small) km |= __ballot(x <= 3);
  }
  return km;
}

template <int T, int BLOCK>
__device__ void flush_stage(SieveShKeys<T, BLOCK>& sh, const SieveParams& P) {
  __syncthreads();
  const uint32_t n = min(sh.stage_n, static_cast<uint32_t>(SieveShKeys<T, BLOCK>::kStage));  // later slots went straight out
  const uint64_t cap1 = P.cap1, W = gridDim.x;
  Entry* l1 = P.l1 + static_cast<uint64_t>(blockIdx.x) * cap1;
  const uint16_t* sb = sh.sb;
  auto* fs = sh.flush_scratch();
  scatter_runs<BLOCK, kB1Max, SieveShKeys<T, BLOCK>::kStage, true>(
      n, P.b1mask + 1, sh.stage, [=](uint32_t i) -> uint32_t { return sb[i]; }, fs->perm, fs->cnt, fs->gofs, sh.wsum,
      sh.lcur, cap1, &P.flags[kFlagL1Overflow],
      [=](uint32_t b, uint32_t k, const Entry& e) { l1[b * W * cap1 + k] = e; }, [] {});
  if (threadIdx.x == 0) sh.stage_n = 0;
  __syncthreads();
}

template <int T, int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) void k_sieve(SieveParams P) {
  using Sh = typename SieveShSel<T, BLOCK, MODE>::type;
  constexpr uint32_t kHitCap = hit_cap<T>();
  static_assert(T % BLOCK == 0 && T <= 65536, "tile shape");
  constexpr int ITER = T / BLOCK;                                     // keys per thread per tile
  constexpr int SLOTS = (dense_slot_cap(T) + BLOCK - 1) / BLOCK;      // dense slots per thread
  static_assert(kDenseMax <= 64 && T / 9 < 1024, "dense slot packing (sdj below)");
  __shared__ Sh sh;
  const int tid = threadIdx.x;
  const DenseTab* D = P.dense;
  const uint32_t nd = D->n, nslots = D->nslots;
  for (uint32_t i = tid; i < nd; i += BLOCK) {
    sh.dq[i] = D->q[i];
    sh.dtq[i] = static_cast<uint32_t>(T) % D->q[i];
  }
  // The dense schedule is the same for every tile: each thread keeps its
  // slots (power index, multiple index, q, p, p^-1) in registers.
  // sdj = d | j << 6 | p << 16 (d < kDenseMax = 64, j <= T / 9 < 1024,
  // p <= sqrt(T) < 2^16), packed to leave registers to the tile loop.
  uint32_t sdj[SLOTS], sq[SLOTS], spinv[SLOTS];
#pragma unroll
  for (int k = 0; k < SLOTS; ++k) {
    const uint32_t t = tid + k * BLOCK;
    if (t < nslots) {
      const uint32_t d = D->slot_d[t];
      sdj[k] = d | ((t - D->prefix[d]) << 6) | (D->p[d] << 16);
      sq[k] = D->q[d];
      spinv[k] = D->pinv[d];
    } else {
      sdj[k] = 1u << 16;
      sq[k] = 0;  // no slot
      spinv[k] = 1;
    }
  }
  if (tid == 0) {
    sh.stage_n = 0;
  }
  if constexpr (MODE == MODE_KEYS) {
    for (uint32_t b = tid; b < kB1Max; b += BLOCK) sh.lcur[b] = 0;
  }
  __syncthreads();
  uint64_t* spill = P.spill + static_cast<uint64_t>(blockIdx.x) * P.spill_cap;

  for (uint64_t s = blockIdx.x; s < P.n_segs; s += gridDim.x) {
    // Segment s -> query q and its x-interval [start, start + len).
    uint32_t lo = 0, hi = P.n_queries;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (P.seg_prefix[mid] <= s)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t qi = lo;
    const uint64_t qa = P.queries[qi].a, qb = P.queries[qi].b;
    const uint64_t start = qa + (s - P.seg_prefix[qi]) * static_cast<uint64_t>(P.seg_len);
    const uint32_t len = static_cast<uint32_t>(min(static_cast<uint64_t>(P.seg_len), qb - start));
    const uint64_t V = start + len;  // largest value sieved in this segment
    // Every tile starts at x0 = qa (mod T) (segments and tiles are multiples
    // of T), so the factor-2 shift of x = x0 + j, j = it * BLOCK + tid, is
    // max(ctz(m), 1) - 1 with m = (qa + j) mod T, the same in every tile,
    // except at the one j with m = 0 (ctz(x) >= log2 T), taken exactly.
    // Four bits per integer of this thread.
    const uint32_t c2 = static_cast<uint32_t>(qa) & static_cast<uint32_t>(T - 1);
    const uint32_t sp_j = (static_cast<uint32_t>(T) - c2) & static_cast<uint32_t>(T - 1);
    uint32_t shifts = 0;
    if constexpr (MODE == MODE_KEYS) {
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const uint32_t m = (c2 + static_cast<uint32_t>(it * BLOCK + tid)) & static_cast<uint32_t>(T - 1);
        const uint32_t tz = m ? static_cast<uint32_t>(__builtin_ctz(m)) : 1u;
        shifts |= (max(tz, 1u) - 1u) << (4 * it);
      }
    }
    // Member test below b/2: y * M <= b fails for every y of the segment when
    // M > lim_hi and holds for every y when M <= lim_lo (y in [start, V]);
    // only M in between needs the exact product.  Both limits are
    // conservative roundings of double quotients.
    uint64_t lim_hi = 0, lim_lo = 0;
    if (MODE == MODE_KEYS && P.prune) {
      const double bd = static_cast<double>(qb);
      lim_hi = static_cast<uint64_t>(bd / static_cast<double>(start > 0 ? start : 1) * (1.0 + 1e-9)) + 1;
      lim_lo = static_cast<uint64_t>(bd / static_cast<double>(V) * (1.0 - 1e-9));
    }
    if (tid == 0) {
      uint32_t l = P.n_dense, h = P.n_pp;
      while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if (P.pp[m].q <= V)
          l = m + 1;
        else
          h = m;
      }
      sh.n_act = l;
      sh.hit_n = 0;
    }
    if (static_cast<uint32_t>(tid) < nd) sh.dres[tid] = static_cast<uint32_t>(start % sh.dq[tid]);
    __syncthreads();

    // Sparse prime powers (q > tile): at most one multiple per tile.  Their
    // multiples in [start, V] are listed once per segment (Algorithm 1's
    // first-multiple offset, start mod q).
    const uint32_t n_act = sh.n_act;
    // Four powers per thread and round, their table words loaded together
    // (a thread past the end loads the last active power and ignores it).
    constexpr int kA = 4;
    for (uint32_t idx0 = P.n_dense + tid; idx0 < n_act; idx0 += kA * BLOCK) {
      PrimePow pw[kA];
#pragma unroll
      for (int u = 0; u < kA; ++u) {
        const uint32_t idx = idx0 + u * BLOCK;
        pw[u] = P.pp[idx < n_act ? idx : n_act - 1];
      }
#pragma unroll
      for (int u = 0; u < kA; ++u) {
        if (idx0 + u * BLOCK >= n_act) break;
        const uint64_t r = mod_fp64(start, pw[u].q, pw[u].invq);
        for (uint64_t j = r ? pw[u].q - r : 0; j <= len; j += pw[u].q) {
          const uint32_t k = atomicAdd(&sh.hit_n, 1u);
          const uint64_t e = (j << 32) | pw[u].p;
          if (k < kHitCap)
            sh.hits[k] = e;
          else if (k - kHitCap < P.spill_cap)
            spill[k - kHitCap] = e;
          else
            atomicOr(&P.flags[kFlagSpillOverflow], 1u);
        }
      }
    }
    __syncthreads();
    const uint32_t nh = min(sh.hit_n, kHitCap + P.spill_cap);

    for (uint32_t base = 0; base < len; base += T) {
      if constexpr (MODE == MODE_KEYS) {
        // Written out once less than the margin is free; stage_n is stable
        // here (after the previous barrier), so the decision is uniform.
        const uint32_t sn = __builtin_amdgcn_readfirstlane(sh.stage_n);
        if (sn > static_cast<uint32_t>(Sh::kStage - Sh::kMargin)) flush_stage<T, BLOCK>(sh, P);
      }
      const uint32_t cnt = min(static_cast<uint32_t>(T), len - base);
      const uint64_t x0 = start + base;
      // r[n] <- n with the prime 2 already reduced (count trailing zeros).
      // The whole tile is written (values past cnt are never used).
      if constexpr (MODE == MODE_KEYS) {
#pragma unroll
        for (int it = 0; it < ITER; ++it)
          sh.tile[it * BLOCK + tid] = (x0 + it * BLOCK + tid) >> ((shifts >> (4 * it)) & 15u);
        if (static_cast<uint32_t>(tid) == (sp_j & static_cast<uint32_t>(BLOCK - 1))) sh.tile[sp_j] = strip_two(x0 + sp_j);
        if (tid == 0) sh.tile[T] = strip_two(x0 + T);
      } else if (const uint32_t x0lo = static_cast<uint32_t>(x0);
                 x0lo != 0u && x0lo <= 0xFFFFFFFFu - static_cast<uint32_t>(T)) {
        // Uniform: no x of the tile (x0 .. x0 + T) has a zero low word.
#pragma unroll
        for (int it = 0; it < ITER; ++it) sh.tile[it * BLOCK + tid] = strip_two_lo(x0 + it * BLOCK + tid);
        if (tid == 0) sh.tile[T] = strip_two_lo(x0 + T);
      } else {
#pragma unroll
        for (int it = 0; it < ITER; ++it) sh.tile[it * BLOCK + tid] = strip_two(x0 + it * BLOCK + tid);
        if (tid == 0) sh.tile[T] = strip_two(x0 + T);
      }
      // dres[d] = x0 mod q_d, advanced by T mod q_d from tile to tile.
      if (static_cast<uint32_t>(tid) < nd) {
        const uint32_t qd = sh.dq[tid];
        uint32_t r = sh.dres[tid];
        if (base) {
          r += sh.dtq[tid];
          if (r >= qd) r -= qd;
          sh.dres[tid] = r;
        }
        sh.doff[tid] = r ? qd - r : 0u;
      }
      __syncthreads();
      // Dense odd prime powers: divide r by p at every multiple of q = p^k.
#pragma unroll
      for (int k = 0; k < SLOTS; ++k) {
        if (sq[k] == 0) continue;
        const uint32_t pos = sh.doff[sdj[k] & 63u] + ((sdj[k] >> 6) & 1023u) * sq[k];
        if (pos <= cnt) lds_div(&sh.tile[pos], sdj[k] >> 16, spinv[k]);
      }
      // Sparse hits of this tile: the LDS list, then the rare spill.
      const uint32_t nh_lds = min(nh, kHitCap);
      for (uint32_t h = tid; h < nh_lds; h += BLOCK) {
        const uint64_t e = sh.hits[h];
        const uint32_t pos = static_cast<uint32_t>(e >> 32);
        if (pos >= base && pos <= base + cnt) {
          const uint32_t p = static_cast<uint32_t>(e);
          lds_div(&sh.tile[pos - base], p, inv32(p));
        }
      }
      for (uint32_t h = kHitCap + tid; h < nh; h += BLOCK) {
        const uint64_t e = spill[h - kHitCap];
        const uint32_t pos = static_cast<uint32_t>(e >> 32);
        if (pos >= base && pos <= base + cnt) {
          const uint32_t p = static_cast<uint32_t>(e);
          lds_div(&sh.tile[pos - base], p, inv32(p));
        }
      }
      __syncthreads();

      if constexpr (MODE == MODE_RAD) {
        for (uint32_t i = tid; i < cnt; i += BLOCK) {
          const uint64_t x = x0 + i;
          if (x >= P.rad_lo && x < P.rad_hi) P.rad_out[x - P.rad_lo] = sh.tile[i];
        }
      } else {
        const uint32_t grp = P.batch ? qi : 0u;
        // Above b/2 no squarefree x or x + 1 passes the member test (the
        // factor t is at least 2): only both-non-squarefree x remain.
        const bool upper = x0 > 3 && x0 > (qb >> 1);
        // 1. The member and pass tests for this thread's ITER integers (cheap,
        // every x).  The tile holds T + 1 values, so the loads need no guard;
        // every branch below is uniform over the wave.
        uint64_t ra[ITER], rb[ITER];
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
          const uint32_t i = it * BLOCK + tid;
          ra[it] = sh.tile[i];
          rb[it] = sh.tile[i + 1];
        }
        // Lane masks of the wave (all 64 lanes are active here): bit l of
        // mask[it] says whether lane l keeps its it-th integer.  The common
        // cases (member test on, one pass, a whole tile) run loops of their
        // own, so that no uniform flag is tested per integer.
        uint64_t mask[ITER];
        uint32_t total = 0;
        const bool full = cnt == static_cast<uint32_t>(T);
        const bool small = x0 <= 3;
        if (P.prune && !P.pfilter && full && upper) {
#pragma unroll
          for (int it = 0; it < ITER; ++it) {
            mask[it] = member_mask<true>(x0 + it * BLOCK + tid, ra[it], rb[it], lim_hi, lim_lo, qb, small);
            total += __popcll(mask[it]);
          }
        } else if (P.prune && !P.pfilter && full) {
#pragma unroll
          for (int it = 0; it < ITER; ++it) {
            mask[it] = member_mask<false>(x0 + it * BLOCK + tid, ra[it], rb[it], lim_hi, lim_lo, qb, small);
            total += __popcll(mask[it]);
          }
        } else {
#pragma unroll
          for (int it = 0; it < ITER; ++it) {
            const uint32_t i = it * BLOCK + tid;
            const uint64_t r0 = ra[it], r1 = rb[it];
            const uint64_t x = x0 + i;
            uint64_t km = ~0ull;
            if (P.prune)
              km = upper ? member_mask<true>(x, r0, r1, lim_hi, lim_lo, qb, small)
                         : member_mask<false>(x, r0, r1, lim_hi, lim_lo, qb, small);
            if (P.pfilter) {
              const uint64_t ph = pass_hash(r0 < r1 ? r0 : r1, r0 < r1 ? r1 : r0, grp);
              km &= __ballot(ph >= P.ph_lo && ph < P.ph_hi);
            }
            if (!full) km &= __ballot(i < cnt);
            mask[it] = km;
            total += __popcll(km);
          }
        }
        // 2. Wave-local compaction: ballots rank the wave's kept integers,
        // lane 0 reserves their stage slots with one LDS atomic, and each
        // kept integer writes its tile index into its slot (two bytes, the
        // only work done per integer with lanes masked off).  The wave then
        // builds the entries of its slots, one slot per lane, from rad(x)
        // and rad(x + 1) still in the tile.  Slots past the stage (a tile
        // that keeps more than the margin left free) are built at once and
        // go straight to the workgroup's regions.
        if (total) {  // uniform over the wave
          const uint64_t below = (1ull << lane_id()) - 1ull;
          uint32_t sbase = 0;
          if (lane_id() == 0) sbase = atomicAdd(&sh.stage_n, total);
          sbase = __builtin_amdgcn_readfirstlane(sbase);
          const uint32_t send = min(sbase + total, static_cast<uint32_t>(Sh::kStage));
          uint32_t sl = sbase;
          if (sbase + total <= static_cast<uint32_t>(Sh::kStage)) {  // the common case: all in the stage
#pragma unroll
            for (int it = 0; it < ITER; ++it) {
              if ((mask[it] >> lane_id()) & 1ull)
                sh.sb[sl + __popcll(mask[it] & below)] = static_cast<uint16_t>(it * BLOCK + tid);
              sl += __popcll(mask[it]);
            }
          } else {
#pragma unroll
            for (int it = 0; it < ITER; ++it) {
              if ((mask[it] >> lane_id()) & 1ull) {
                const uint32_t i = it * BLOCK + tid;
                const uint32_t slot = sl + __popcll(mask[it] & below);
                if (slot < static_cast<uint32_t>(Sh::kStage)) {
                  sh.sb[slot] = static_cast<uint16_t>(i);
                } else {
                  uint32_t bk;
                  const Entry e = kept_entry(P, ra[it], rb[it], x0 + i, qa, grp, &bk);
                  const uint32_t g = atomicAdd(&sh.lcur[bk], 1u);
                  if (g < P.cap1)
                    P.l1[(static_cast<uint64_t>(bk) * gridDim.x + blockIdx.x) * P.cap1 + g] = e;
                  else
                    atomicOr(&P.flags[kFlagL1Overflow], 1u);
                }
              }
              sl += __popcll(mask[it]);
            }
          }
          wave_sync();
          for (uint32_t sidx = sbase + lane_id(); sidx < send; sidx += 64) {
            const uint32_t i = sh.sb[sidx];
            uint32_t bk;
            sh.stage[sidx] = kept_entry(P, sh.tile[i], sh.tile[i + 1], x0 + i, qa, grp, &bk);
            sh.sb[sidx] = static_cast<uint16_t>(bk);
          }
        }
      }
      __syncthreads();
    }
  }
  if constexpr (MODE == MODE_KEYS) {
    __syncthreads();
    const uint32_t sn = __builtin_amdgcn_readfirstlane(sh.stage_n);
    if (sn > 0) flush_stage<T, BLOCK>(sh, P);
    for (uint32_t b = tid; b <= P.b1mask; b += BLOCK) P.cnt1[static_cast<uint64_t>(b) * gridDim.x + blockIdx.x] = sh.lcur[b];
  }
}

struct PartParams {
  const Entry* l1;
  uint64_t cap1;          // entries per first-level region
  const uint32_t* cnt1;   // B1 x W region fill counts
  uint32_t W;             // regions per bucket (sieve workgroups)
  uint32_t first;  // first first-level bucket of this group
  uint32_t G;      // buckets in the group: 1, 2, 4 or 8
  uint32_t chunks_per_region;
  Entry* l2;       // group buffer: G x B2 sub-buckets of cap2 entries
  uint32_t cap2;
  uint32_t* cnt2;  // G x B2 cursors (zero on entry)
  uint32_t b2shift, b2mask;  // second-level partition = top bits of the fingerprint
  uint64_t fp_mask;          // fingerprint bits kept (all 53 but in tests of the verification)
  uint32_t gmask;
  uint32_t* flags;
  // Compact second level: one 64-bit word per entry, fp_low << idx_bits | i,
  // with i = w * cap1 + k the entry's index among its first-level bucket's
  // regions (entry k of region (b, w)), which stay intact until the group is
  // joined.  The top of the fingerprint is the partition's own index.
  uint64_t* l2c;
  uint32_t idx_bits;
  uint64_t low_mask;  // fingerprint bits a compact word keeps
};

__device__ __forceinline__ uint64_t compact_word(const PartParams& P, const Entry& e, uint64_t idx) {
  return ((entry_fp(e) & P.low_mask) << P.idx_bits) | idx;
}

// Second scatter of one group of first-level buckets into the group buffer.
// Persistent: workgroup l runs on XCD l mod 8 (round-robin dispatch) and
// serves bucket (l mod 8) mod G, so with G = 8 a bucket never leaves its XCD
// and the partial lines of its sub-buckets are completed in that XCD's L2
// before they are written back.  The bucket's chunks are split into nbw
// contiguous ranges, one per workgroup; the next chunk is loaded into
// registers while the current one is scattered.
template <int BLOCK, bool MASK_FP, bool COMPACT>
__global__ __launch_bounds__(BLOCK) void k_partition(PartParams P) {
  constexpr int EPT = kPartChunk / BLOCK;
  static_assert(kPartChunk % BLOCK == 0, "chunk shape");
  using Item = typename std::conditional<COMPACT, uint64_t, Entry>::type;  // what the chunk stages
  __shared__ Item ent[kPartChunk];
  __shared__ uint16_t sbk[kPartChunk], perm[kPartChunk];
  __shared__ uint32_t cnt[kB2Max], gofs[kB2Max];
  __shared__ uint32_t wsum[BLOCK / 64];
  const int tid = threadIdx.x;
  const uint32_t l = blockIdx.x;
  const uint32_t xcd = l & 7u, slot = l >> 3;
  const uint32_t per = 8u / P.G;
  const uint32_t gb = xcd % P.G;
  const uint32_t k = slot * per + xcd / P.G;  // index among the bucket's nbw workgroups
  const uint32_t nbw = (gridDim.x >> 3) * per;
  const uint32_t b1 = P.first + gb;
  const uint32_t B2 = P.b2mask + 1;
  const uint32_t cpr = P.chunks_per_region;
  const uint64_t n_chunks = static_cast<uint64_t>(P.W) * cpr;
  const uint64_t c_begin = n_chunks * k / nbw, c_end = n_chunks * (k + 1) / nbw;
  Entry* out = P.l2 + static_cast<uint64_t>(gb) * B2 * P.cap2;
  uint64_t* outc = P.l2c + static_cast<uint64_t>(gb) * B2 * P.cap2;
  uint32_t* gcur = P.cnt2 + static_cast<uint64_t>(gb) * B2;
  const uint32_t cap2 = P.cap2;
  // The partition of an entry is the top of its fingerprint.
  auto bucket_of = [&](uint32_t i) -> uint32_t { return sbk[i]; };
  // Chunk ci of the bucket: entries [s0, s0 + n) of region ci / cpr.
  auto chunk = [&](uint64_t ci, const Entry** src) -> uint32_t {  // ci < n_chunks
    const uint64_t region = static_cast<uint64_t>(b1) * P.W + ci / cpr;
    const uint64_t n1 = min(static_cast<uint64_t>(P.cnt1[region]), P.cap1);
    const uint64_t s0 = (ci % cpr) * static_cast<uint64_t>(kPartChunk);
    *src = P.l1 + region * P.cap1 + s0;
    return s0 >= n1 ? 0u : static_cast<uint32_t>(min(static_cast<uint64_t>(kPartChunk), n1 - s0));
  };
  Entry e[EPT];
  const Entry* src;
  uint32_t n = c_begin < c_end ? chunk(c_begin, &src) : 0u;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const uint32_t i = tid + q * BLOCK;
    if (i < n) e[q] = src[i];
  }
  for (uint64_t ci = c_begin; ci < c_end; ++ci) {
    // Index of the chunk's first entry among the bucket's regions (compact words).
    const uint64_t ibase = COMPACT ? (ci / cpr) * P.cap1 + (ci % cpr) * static_cast<uint64_t>(kPartChunk) : 0ull;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const uint32_t i = tid + q * BLOCK;
      if (i < n) {
        Entry x = e[q];
        if constexpr (MASK_FP) {  // tests of the verification only
          const uint64_t pos43 = entry_pos43(x);
          x = make_entry(pos43, entry_fp(x) & P.fp_mask);
        }
        if constexpr (COMPACT)
          ent[i] = compact_word(P, x, ibase + i);
        else
          ent[i] = x;
        sbk[i] = static_cast<uint16_t>(static_cast<uint32_t>(entry_fp(e[q]) >> P.b2shift) & P.b2mask);
      }
    }
    const uint32_t n_cur = n;
    n = ci + 1 < c_end ? chunk(ci + 1, &src) : 0u;
    // Issued after the global cursor atomics, whose returns would otherwise
    // wait for these loads as well.
    auto prefetch = [&] {
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const uint32_t i = tid + q * BLOCK;
        if (i < n) e[q] = src[i];
      }
    };
    __syncthreads();
    if (n_cur)  // uniform over the workgroup
      scatter_runs<BLOCK, kB2Max, kPartChunk, false>(
          n_cur, B2, ent, bucket_of, perm, cnt, gofs, wsum, gcur, cap2, &P.flags[kFlagL2Overflow],
          [=](uint32_t b, uint32_t kk, const Item& x) {
            if constexpr (COMPACT)
              outc[static_cast<uint64_t>(b) * cap2 + kk] = x;
            else
              out[static_cast<uint64_t>(b) * cap2 + kk] = x;
          },
          prefetch);
    else
      prefetch();
  }
}

struct JoinParams {
  const Entry* l2;
  uint32_t cap2;
  uint32_t* cnt2;
  uint64_t n_sub;
  uint32_t gmask;
  Cand* cand;
  uint32_t cand_cap;
  uint32_t* flags;
  unsigned long long* joined;  // entries read, summed over partitions (64-bit: 2^36 searches pass 2^32)
  // Compact second level (k_join_c): the words and the first level they index.
  const uint64_t* l2c;
  uint32_t idx_bits;
  const Entry* l1;
  uint64_t cap1;
  uint32_t W, first;  // regions per bucket; first first-level bucket of the group
  uint32_t b2mask;    // sub-bucket sbk is partition sbk & b2mask of bucket first + sbk / (b2mask + 1)
};

// The 12-byte entry a compact word of sub-bucket sbk stands for, read back
// from its first-level region.
__device__ __forceinline__ Entry compact_entry(const JoinParams& P, uint64_t w, uint64_t sbk) {
  const uint64_t b1 = P.first + sbk / (static_cast<uint64_t>(P.b2mask) + 1);
  return P.l1[b1 * P.W * P.cap1 + (w & ((1ull << P.idx_bits) - 1))];
}

__device__ __forceinline__ void emit_cand(const JoinParams& P, const Entry& a, const Entry& b) {
  const uint32_t k = atomicAdd(&P.flags[kFlagCand], 1u);
  if (k < P.cand_cap) {
    Cand c;
    c.a = a;
    c.b = b;
    P.cand[k] = c;
  }
}

// LDS hash join of one second-level partition.  Each insert walks its probe
// chain to the first empty slot and compares the key with every occupied slot
// on the way (Algorithm 3's insert step).  Two equal keys follow the same
// chain, so the one that claims the later slot passes the other and reports
// the pair; every pair of a group is reported once.  A slot holds an 18-bit
// tag of the key hash and the entry's index; the entries themselves stay in
// registers (EPT per thread), and the rare tag match re-reads the other entry
// from the partition (L2-resident).  Partitions larger than one chunk are
// joined chunk by chunk: after chunk c is inserted, every later entry probes
// it, walking to an empty slot as the probe step does.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_join(JoinParams P) {
  constexpr int EPT = kJoinCap / BLOCK;
  constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  constexpr uint32_t kIdxMask = (1u << kJoinIdxBits) - 1;
  static_assert(kJoinCap < (1 << kJoinIdxBits), "index field must not reach the empty marker");
  __shared__ __align__(16) uint32_t table[kJoinSlots];
  const int tid = threadIdx.x;
  const uint64_t sbk = blockIdx.x;
  if (sbk >= P.n_sub) return;
  const uint32_t n = min(P.cnt2[sbk], P.cap2);
  __syncthreads();
  // This workgroup is the only reader of the cursor: clear it for the next group.
  if (tid == 0) {
    P.cnt2[sbk] = 0;
    if (n) atomicAdd(P.joined, static_cast<unsigned long long>(n));
  }
  if (n < 2) return;
  const Entry* src = P.l2 + sbk * P.cap2;
  for (uint32_t i0 = 0; i0 < n; i0 += kJoinCap) {
    const uint32_t m = min(static_cast<uint32_t>(kJoinCap), n - i0);
    // Table of at least twice the chunk's entries (load <= 0.5), power of two.
    uint32_t slots = 1024;
    while (slots < 2 * m && slots < static_cast<uint32_t>(kJoinSlots)) slots <<= 1;
    const uint32_t smask = slots - 1;
    // Every thread loads all its entries at once: lanes past the chunk load
    // entry 0 instead (m >= 2), so that no load waits behind a masked one.
    Entry e[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const uint32_t i = tid + k * BLOCK;
      e[k] = src[i0 + (i < m ? i : 0u)];
    }
    // Cleared four slots per store (slots is a multiple of 1024).
    for (uint32_t s = 4 * tid; s < slots; s += 4 * BLOCK)
      *reinterpret_cast<uint4*>(&table[s]) = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    __syncthreads();
    // Every entry first tries to claim its home slot; the EPT claims of a
    // thread are independent and issued together (at load <= 0.5 most
    // succeed).  A claim that finds the slot taken compares the tag and walks
    // on, claiming each next slot, until one is empty.
    // (In groups of four, to stay within the registers of 32 waves per CU.)
    constexpr int kClaim = EPT < 4 ? EPT : 4;
    static_assert(EPT % kClaim == 0, "claim groups");
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += kClaim) {
      uint32_t got[kClaim];
#pragma unroll
      for (int u = 0; u < kClaim; ++u) {
        const uint32_t i = tid + (k0 + u) * BLOCK;
        const uint32_t h = static_cast<uint32_t>(entry_fp(e[k0 + u]));
        got[u] = i < m ? atomicCAS(&table[h & smask], kEmpty, (h & ~kIdxMask) | i) : kEmpty;
      }
#pragma unroll
      for (int u = 0; u < kClaim; ++u) {
        if (got[u] == kEmpty) continue;  // claimed (or no entry)
        const int k = k0 + u;
        const uint64_t fk = entry_fp(e[k]);
        const uint32_t gk = entry_grp(e[k], P.gmask);
        const uint32_t h = static_cast<uint32_t>(fk);
        const uint32_t mine = (h & ~kIdxMask) | (tid + k * BLOCK);
        uint32_t v = got[u], s = h & smask;
        for (;;) {
          if (((v ^ mine) & ~kIdxMask) == 0) {
            const Entry f = src[i0 + (v & kIdxMask)];
            if (entry_fp(f) == fk && entry_grp(f, P.gmask) == gk) emit_cand(P, e[k], f);
          }
          s = (s + 1) & smask;
          v = atomicCAS(&table[s], kEmpty, mine);
          if (v == kEmpty) break;
        }
      }
    }
    __syncthreads();
    for (uint32_t jj = i0 + m + tid; jj < n; jj += BLOCK) {
      const Entry g = src[jj];
      const uint64_t fk = entry_fp(g);
      const uint32_t gk = entry_grp(g, P.gmask);
      const uint32_t h = static_cast<uint32_t>(fk);
      uint32_t s = h & smask;
      for (;;) {
        const uint32_t v = table[s];
        if (v == kEmpty) break;
        if (((v ^ h) & ~kIdxMask) == 0) {
          const Entry f = src[i0 + (v & kIdxMask)];
          if (entry_fp(f) == fk && entry_grp(f, P.gmask) == gk) emit_cand(P, g, f);
        }
        s = (s + 1) & smask;
      }
    }
    __syncthreads();
  }
}

// k_join over compact words: the same inserts and probes, on the kept low
// fingerprint bits (the partition fixes the top ones).  Both entries of a
// match are read back from the first level and become a candidate when their
// whole fingerprints and queries agree, as in k_join.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_join_c(JoinParams P) {
  constexpr int EPT = kJoinCap / BLOCK;
  constexpr uint32_t kEmpty = 0xFFFFFFFFu;
  constexpr uint32_t kIdxMask = (1u << kJoinIdxBits) - 1;
  static_assert(kJoinCap < (1 << kJoinIdxBits), "index field must not reach the empty marker");
  __shared__ __align__(16) uint32_t table[kJoinSlots];
  const int tid = threadIdx.x;
  const uint64_t sbk = blockIdx.x;
  if (sbk >= P.n_sub) return;
  const uint32_t n = min(P.cnt2[sbk], P.cap2);
  __syncthreads();
  if (tid == 0) {
    P.cnt2[sbk] = 0;
    if (n) atomicAdd(P.joined, static_cast<unsigned long long>(n));
  }
  if (n < 2) return;
  const uint64_t* src = P.l2c + sbk * P.cap2;
  const uint32_t pb = P.idx_bits;
  auto emit = [&](uint64_t a, uint64_t b) {
    atomicAdd(&P.flags[kFlagWordMatch], 1u);
    const Entry ea = compact_entry(P, a, sbk), eb = compact_entry(P, b, sbk);
    if (entry_fp(ea) == entry_fp(eb) && entry_grp(ea, P.gmask) == entry_grp(eb, P.gmask)) emit_cand(P, ea, eb);
  };
  for (uint32_t i0 = 0; i0 < n; i0 += kJoinCap) {
    const uint32_t m = min(static_cast<uint32_t>(kJoinCap), n - i0);
    uint32_t slots = 1024;
    while (slots < 2 * m && slots < static_cast<uint32_t>(kJoinSlots)) slots <<= 1;
    const uint32_t smask = slots - 1;
    uint64_t e[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const uint32_t i = tid + k * BLOCK;
      e[k] = src[i0 + (i < m ? i : 0u)];
    }
    for (uint32_t s = 4 * tid; s < slots; s += 4 * BLOCK)
      *reinterpret_cast<uint4*>(&table[s]) = make_uint4(kEmpty, kEmpty, kEmpty, kEmpty);
    __syncthreads();
    constexpr int kClaim = EPT < 4 ? EPT : 4;
    static_assert(EPT % kClaim == 0, "claim groups");
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += kClaim) {
      uint32_t got[kClaim];
#pragma unroll
      for (int u = 0; u < kClaim; ++u) {
        const uint32_t i = tid + (k0 + u) * BLOCK;
        const uint32_t h = static_cast<uint32_t>(e[k0 + u] >> pb);
        got[u] = i < m ? atomicCAS(&table[h & smask], kEmpty, (h & ~kIdxMask) | i) : kEmpty;
      }
#pragma unroll
      for (int u = 0; u < kClaim; ++u) {
        if (got[u] == kEmpty) continue;
        const int k = k0 + u;
        const uint64_t fk = e[k] >> pb;
        const uint32_t h = static_cast<uint32_t>(fk);
        const uint32_t mine = (h & ~kIdxMask) | (tid + k * BLOCK);
        uint32_t v = got[u], s = h & smask;
        for (;;) {
          if (((v ^ mine) & ~kIdxMask) == 0) {
            const uint64_t f = src[i0 + (v & kIdxMask)];
            if ((f >> pb) == fk) emit(e[k], f);
          }
          s = (s + 1) & smask;
          v = atomicCAS(&table[s], kEmpty, mine);
          if (v == kEmpty) break;
        }
      }
    }
    __syncthreads();
    for (uint32_t jj = i0 + m + tid; jj < n; jj += BLOCK) {
      const uint64_t g = src[jj];
      const uint64_t fk = g >> pb;
      const uint32_t h = static_cast<uint32_t>(fk);
      uint32_t s = h & smask;
      for (;;) {
        const uint32_t v = table[s];
        if (v == kEmpty) break;
        if (((v ^ h) & ~kIdxMask) == 0) {
          const uint64_t f = src[i0 + (v & kIdxMask)];
          if ((f >> pb) == fk) emit(g, f);
        }
        s = (s + 1) & smask;
      }
    }
    __syncthreads();
  }
}

// Sort join of one second-level partition, the ablation of the LDS hash join:
// Algorithm 2 (sort, then compare neighbours) applied per partition, with every
// pair of a run of equal keys reported rather than adjacent ones only.  The low
// 32 bits of each fingerprint, packed with the entry's index, are bitonic-
// sorted in LDS; runs of equal words are compared on the full fingerprint and
// query.  A partition larger than one LDS chunk is joined chunk by chunk: every
// later entry binary-searches each sorted chunk.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_join_sort(JoinParams P) {
  constexpr int kIdx = 13;  // index bits (kJoinCap = 8192)
  static_assert(kJoinCap <= (1 << kIdx), "index field");
  __shared__ uint64_t key[kJoinCap];
  const int tid = threadIdx.x;
  const uint64_t sbk = blockIdx.x;
  if (sbk >= P.n_sub) return;
  const uint32_t n = min(P.cnt2[sbk], P.cap2);
  __syncthreads();
  // This workgroup is the only reader of the cursor: clear it for the next group.
  if (tid == 0) {
    P.cnt2[sbk] = 0;
    if (n) atomicAdd(P.joined, static_cast<unsigned long long>(n));
  }
  if (n < 2) return;
  const Entry* src = P.l2 + sbk * P.cap2;
  auto same = [&](const Entry& a, const Entry& b) {
    return entry_fp(a) == entry_fp(b) && entry_grp(a, P.gmask) == entry_grp(b, P.gmask);
  };
  for (uint32_t i0 = 0; i0 < n; i0 += kJoinCap) {
    const uint32_t m = min(static_cast<uint32_t>(kJoinCap), n - i0);
    uint32_t npad = 2;
    while (npad < m) npad <<= 1;
    for (uint32_t i = tid; i < npad; i += BLOCK)
      key[i] = i < m ? (static_cast<uint64_t>(static_cast<uint32_t>(entry_fp(src[i0 + i]))) << kIdx) | i : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= npad; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t t = tid; t < npad / 2; t += BLOCK) {
          const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1)), l = i | j;
          const uint64_t a = key[i], b = key[l];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[l] = a;
          }
        }
        __syncthreads();
      }
    }
    // Runs of equal 32-bit fingerprint words inside the chunk: the thread at a
    // run's first element compares every pair of the run in full.
    for (uint32_t i = tid; i + 1 < m; i += BLOCK) {
      const uint64_t h = key[i] >> kIdx;
      if ((i > 0 && (key[i - 1] >> kIdx) == h) || (key[i + 1] >> kIdx) != h) continue;
      uint32_t end = i + 1;
      while (end < m && (key[end] >> kIdx) == h) ++end;
      for (uint32_t a = i; a < end; ++a) {
        const Entry ea = src[i0 + static_cast<uint32_t>(key[a] & ((1u << kIdx) - 1))];
        for (uint32_t b = a + 1; b < end; ++b) {
          const Entry eb = src[i0 + static_cast<uint32_t>(key[b] & ((1u << kIdx) - 1))];
          if (same(ea, eb)) emit_cand(P, ea, eb);
        }
      }
    }
    // Every later entry searches this sorted chunk.
    for (uint32_t jj = i0 + m + tid; jj < n; jj += BLOCK) {
      const Entry g = src[jj];
      const uint64_t h = static_cast<uint32_t>(entry_fp(g));
      uint32_t lo = 0, hi = m;  // first word with key >> kIdx >= h
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((key[mid] >> kIdx) < h)
          lo = mid + 1;
        else
          hi = mid;
      }
      for (uint32_t a = lo; a < m && (key[a] >> kIdx) == h; ++a) {
        const Entry f = src[i0 + static_cast<uint32_t>(key[a] & ((1u << kIdx) - 1))];
        if (same(g, f)) emit_cand(P, g, f);
      }
    }
    __syncthreads();
  }
}

struct VerifyParams {
  const Cand* cand;
  const uint32_t* n_cand;  // candidate count, read on the device (graph replays)
  uint32_t cand_cap;
  const uint32_t* primes;  // all primes <= sqrt(hi_max), ascending
  const PrimeInv* pinv;    // their inverses for the divisibility tests
  uint32_t n_primes;
  const Query* queries;
  int batch;
  uint32_t kinds;
  uint32_t third_off;  // the third condition compares rad(m + third_off), rad(n + third_off) (2 in use)
  uint64_t fp_mask;
  OutPair* out;
  uint32_t out_cap;
  uint32_t* flags;
};

// One workgroup per candidate pair: rad of m, m+1, n, n+1 by trial division
// (the definition of the radical), with the cofactor left after dividing out
// every prime <= sqrt(v) being 1 or one more prime.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_verify(VerifyParams P) {
  constexpr int NV = 6;  // m, m+1, n, n+1 and, for the third condition, m+d, n+d (d = 2)
  __shared__ uint64_t red_r[NV][BLOCK], red_s[NV][BLOCK];
  const int tid = threadIdx.x;
  const uint32_t n_cand = min(*P.n_cand, P.cand_cap);
  const bool third = (P.kinds & kKindThird) != 0;
  const int nv = third ? NV : 4;
  for (uint32_t c = blockIdx.x; c < n_cand; c += gridDim.x) {
    __syncthreads();
    const Cand cd = P.cand[c];
    const uint32_t qa_idx = entry_grp(cd.a, P.batch ? kGrpMask : 0u);
    const uint64_t off = P.batch ? P.queries[qa_idx].a : 0ull;
    const uint64_t xa = entry_pos(cd.a, P.batch) + off, xb = entry_pos(cd.b, P.batch) + off;
    const uint64_t m = xa < xb ? xa : xb, n = xa < xb ? xb : xa;
    const uint64_t d = P.third_off;
    const uint64_t v[NV] = {m, m + 1, n, n + 1, m + d, n + d};
    const uint64_t vmax = third && d > 1 ? n + d : n + 1;
    uint64_t pr[NV] = {1, 1, 1, 1, 1, 1}, sm[NV] = {1, 1, 1, 1, 1, 1};
    for (uint32_t i = tid; i < P.n_primes; i += BLOCK) {
      const uint64_t p = P.primes[i];
      if (p * p > vmax) break;
      if (p == 2) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          if (k < nv && 4 <= v[k] && (v[k] & 1) == 0) {
            pr[k] *= 2;
            sm[k] <<= __builtin_ctzll(v[k]);
          }
        }
        continue;
      }
      // An odd p divides t iff t * p^-1 (mod 2^64) <= floor((2^64 - 1) / p),
      // and that product is then t / p.
      const PrimeInv pi = P.pinv[i];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        uint64_t t = v[k] * pi.inv;
        if (k < nv && p * p <= v[k] && t <= pi.lim) {
          pr[k] *= p;
          uint64_t pk = p;
          for (uint64_t u = t * pi.inv; u <= pi.lim; u *= pi.inv) pk *= p;
          sm[k] *= pk;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      red_r[k][tid] = pr[k];
      red_s[k][tid] = sm[k];
    }
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
      if (tid < w) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          red_r[k][tid] *= red_r[k][tid + w];
          red_s[k][tid] *= red_s[k][tid + w];
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      uint64_t rad[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const uint64_t cof = v[k] / red_s[k][0];
        rad[k] = red_r[k][0] * (cof > 1 ? cof : 1);
      }
      const uint64_t lo_m = rad[0] < rad[1] ? rad[0] : rad[1], hi_m = rad[0] < rad[1] ? rad[1] : rad[0];
      const uint64_t lo_n = rad[2] < rad[3] ? rad[2] : rad[3], hi_n = rad[2] < rad[3] ? rad[3] : rad[2];
      const bool same = (lo_m == lo_n) && (hi_m == hi_n) && m != n &&
                        entry_grp(cd.b, P.batch ? kGrpMask : 0u) == qa_idx;
      if (!same) {
        atomicAdd(&P.flags[kFlagFalseCand], 1u);  // equal fingerprints, different sets (or queries)
      } else if (((key64(lo_m, hi_m, P.batch ? qa_idx : 0u) >> 11) & P.fp_mask) != entry_fp(cd.a)) {
        atomicAdd(&P.flags[kFlagVerifyFail], 1u);  // the entry does not hold this set's fingerprint
      } else {
        // Kind 1 iff rad(m) = rad(n) (Algorithm 2); the third-condition bit
        // marks a first-kind pair with rad(m + 2) = rad(n + 2) as well.
        const uint32_t base = rad[0] == rad[2] ? 1u : 2u;
        const bool three = third && base == 1u && rad[4] == rad[5];
        const uint32_t kind = base | (three ? kKindThird : 0u);
        if ((P.kinds & base) || three) {
          const uint32_t k = atomicAdd(&P.flags[kFlagOut], 1u);
          if (k < P.out_cap) {
            OutPair o;
            o.m = m;
            o.n = n;
            o.kind = kind;
            o.query = P.batch ? qa_idx : 0u;
            P.out[k] = o;
          }
        }
      }
    }
  }
}

// Sum of n counters into *acc (entries written by a pass).
__global__ void k_sum_counts(const uint32_t* cnt, uint64_t n, unsigned long long* acc) {
  uint64_t s = 0;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    s += cnt[i];
  if (s) atomicAdd(acc, static_cast<unsigned long long>(s));
}

// The one-query table of a single-range sieve, written from kernel arguments
// (no host copy).
__global__ void k_set_query(Query* q, uint64_t* seg_prefix, uint64_t a, uint64_t b, uint64_t n_segs) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    q->a = a;
    q->b = b;
    seg_prefix[0] = 0;
    seg_prefix[1] = n_segs;
  }
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

}  // namespace bx
