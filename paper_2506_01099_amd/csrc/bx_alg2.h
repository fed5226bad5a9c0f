// Algorithm 2 of the paper as HIP kernels (a baseline beside the hash-
// partitioned passes): the radicals of the whole range, one list entry
// (S_n, n) per integer n, the list sorted by S_n, and every run of equal keys
// reported.  The sort key is the 53-bit fingerprint of the set
// S_n = {rad(n), rad(n + 1)} (equal sets have equal fingerprints; different
// sets that share one are dropped by the verification, which recomputes the
// radicals).  Where the paper compares neighbours only, every pair inside a
// run is reported, so groups of three or more equal sets give all their pairs.
//
//   k_a2_keys      fingerprints of the kept integers of one chunk of radicals,
//                  compacted into the list (one atomic per tile of 4096).
//   k_rs_hist      least-significant-digit radix sort, 8 bits per pass: digit
//   k_scan_*       counts per tile, an exclusive scan over (digit, tile), and
//   k_rs_scatter   a stable scatter (lanes of a wave rank equal digits by
//                  ballots; waves keep running counts in LDS).
//   k_a2_runs      every pair inside each run of equal keys of the sorted list.
#pragma once
#include "bx_kernels.h"

namespace bx {

constexpr int kRsBlock = 256;                 // threads of a sort workgroup (4 waves)
constexpr int kRsIter = 16;                   // items per thread
constexpr int kRsTile = kRsBlock * kRsIter;   // items per workgroup
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

struct A2KeyParams {
  const uint64_t* rad;  // rad[t] = rad(c0 + t), t in [0, count]
  uint64_t c0;
  uint32_t count;
  uint64_t qb;          // end of the range (member test)
  uint32_t prune;
  uint64_t fp_mask;
  uint64_t* keys;
  uint64_t* vals;
  uint64_t cap;
  unsigned long long* n_out;  // entries written so far (all chunks)
  uint32_t* flags;
};

// One tile of BLOCK * kA2Items consecutive integers per step: each thread
// tests its kA2Items integers (strided by BLOCK, so that the radical loads
// coalesce), a block scan ranks the kept ones, and one atomic per tile
// reserves their list entries (one counter shared by the whole grid, so the
// reservations must be few).
constexpr int kA2Items = 16;
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_a2_keys(A2KeyParams P) {
  __shared__ uint32_t wsum[BLOCK / 64];
  __shared__ unsigned long long base_s;
  constexpr uint64_t kTileN = static_cast<uint64_t>(BLOCK) * kA2Items;
  for (uint64_t t0 = blockIdx.x * kTileN; t0 < P.count; t0 += gridDim.x * kTileN) {
    uint32_t keep = 0;
    uint64_t fp[kA2Items];
#pragma unroll
    for (int k = 0; k < kA2Items; ++k) {
      const uint64_t t = t0 + static_cast<uint64_t>(k) * BLOCK + threadIdx.x;
      fp[k] = 0;
      if (t < P.count) {
        const uint64_t r0 = P.rad[t], r1 = P.rad[t + 1];
        if (!P.prune || may_pair(P.c0 + t, r0, r1, P.qb)) {
          keep |= 1u << k;
          fp[k] = (key64(r0 < r1 ? r0 : r1, r0 < r1 ? r1 : r0, 0) >> 11) & P.fp_mask;
        }
      }
    }
    uint32_t total = 0;
    const uint32_t pre = block_exclusive_scan<BLOCK>(static_cast<uint32_t>(__popc(keep)), wsum, &total);
    if (threadIdx.x == 0) base_s = total ? atomicAdd(P.n_out, static_cast<unsigned long long>(total)) : 0ull;
    __syncthreads();
    uint64_t k_out = base_s + pre;
    __syncthreads();  // base_s and wsum are rewritten by the next tile
#pragma unroll
    for (int k = 0; k < kA2Items; ++k) {
      if ((keep >> k) & 1u) {
        if (k_out < P.cap) {
          P.keys[k_out] = fp[k];
          P.vals[k_out] = P.c0 + t0 + static_cast<uint64_t>(k) * BLOCK + threadIdx.x;
        } else {
          atomicOr(&P.flags[kFlagL1Overflow], 1u);
        }
        ++k_out;
      }
    }
  }
}

// Digit counts of tile b: hist[d * n_tiles + b] (digit-major, so that the
// exclusive scan gives every (digit, tile) its first output position).
__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const uint64_t* keys, uint64_t n, uint32_t shift, uint32_t* hist,
                                                     uint64_t n_tiles) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint64_t base = blockIdx.x * static_cast<uint64_t>(kRsTile);
#pragma unroll
  for (int it = 0; it < kRsIter; ++it) {
    const uint64_t i = base + it * kRsBlock + tid;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[tid * n_tiles + blockIdx.x] = h[tid];
}

// Exclusive scan of m 32-bit counts into 64-bit offsets, in three steps:
// tiles of kScanTile (local scan, tile totals), the totals, the carry-in.
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const uint32_t* in, uint64_t m, uint64_t* out,
                                                          uint64_t* totals) {
  __shared__ uint64_t wsum[kScanBlock / 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint64_t base = blockIdx.x * static_cast<uint64_t>(kScanTile) + static_cast<uint64_t>(tid) * kScanItems;
  uint64_t v[kScanItems], s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < m ? in[base + k] : 0u;
    s += v[k];
  }
  uint64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint64_t w = lane < kScanBlock / 64 ? wsum[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < kScanBlock / 64) wsum[lane] = w;
  }
  __syncthreads();
  uint64_t run = (wid ? wsum[wid - 1] : 0) + x - s;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < m) out[base + k] = run;
    run += v[k];
  }
  if (tid == kScanBlock - 1) totals[blockIdx.x] = wsum[kScanBlock / 64 - 1];
}

// One workgroup: exclusive scan of the nt tile totals, in place.
__global__ __launch_bounds__(kScanBlock) void k_scan_totals(uint64_t* totals, uint64_t nt) {
  __shared__ uint64_t wsum[kScanBlock / 64];
  __shared__ uint64_t carry_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (uint64_t b0 = 0; b0 < nt; b0 += kScanBlock) {
    const uint64_t i = b0 + tid;
    const uint64_t v = i < nt ? totals[i] : 0;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
      uint64_t w = lane < kScanBlock / 64 ? wsum[lane] : 0;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(w, o, 64);
        if (lane >= o) w += y;
      }
      if (lane < kScanBlock / 64) wsum[lane] = w;
    }
    __syncthreads();
    const uint64_t carry = carry_s;
    if (i < nt) totals[i] = carry + (wid ? wsum[wid - 1] : 0) + x - v;
    __syncthreads();
    if (tid == 0) carry_s = carry + wsum[kScanBlock / 64 - 1];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(uint64_t* out, uint64_t m, const uint64_t* totals) {
  const uint64_t base = blockIdx.x * static_cast<uint64_t>(kScanTile);
  const uint64_t add = totals[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k * kScanBlock + threadIdx.x;
    if (i < m) out[i] += add;
  }
}

// Stable scatter of tile b by the digit at `shift`.  Wave w owns the items
// [w * 1024, (w + 1) * 1024) of the tile, 64 consecutive items per step, so
// index order is (wave, step, lane) order.  Lanes holding the same digit find
// each other with eight ballots; the group's first lane advances the wave's
// running count of that digit.  The tile is then sorted by digit in LDS
// (keys, then values, through one staging array) and written out with
// consecutive threads on consecutive positions of each digit's run: the
// digit's run starts at the scanned offset of (digit, tile).
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const uint64_t* keys_in, const uint64_t* vals_in, uint64_t n,
                                                        uint32_t shift, const uint64_t* offs, uint64_t n_tiles,
                                                        uint64_t* keys_out, uint64_t* vals_out) {
  constexpr int W = kRsBlock / 64;
  static_assert(kRsBlock == 256, "one thread per digit below");
  __shared__ uint32_t wc[W][256];   // running counts, then each (wave, digit)'s first tile position
  __shared__ uint32_t tstart[256];  // first tile position of each digit
  __shared__ uint64_t gofs[256];    // first output position of each digit's run
  __shared__ uint32_t wsum[W];
  __shared__ uint64_t stage[kRsTile];
  __shared__ uint8_t sdig[kRsTile];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < W; ++k) wc[k][tid] = 0;
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;
  const uint64_t tile0 = blockIdx.x * static_cast<uint64_t>(kRsTile);
  const uint64_t base = tile0 + static_cast<uint64_t>(w) * (kRsTile / W);
  uint64_t key[kRsIter];
  uint32_t pos[kRsIter];  // rank among the wave's equal digits, then the tile position
#pragma unroll
  for (int it = 0; it < kRsIter; ++it) {
    const uint64_t i = base + it * 64 + lane;
    const bool ok = i < n;
    key[it] = ok ? keys_in[i] : 0;
    const uint32_t d = static_cast<uint32_t>(key[it] >> shift) & 255u;
    uint64_t same = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1u);
      same &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t c0 = wc[w][d];
    if (ok && (same & below) == 0) wc[w][d] = c0 + static_cast<uint32_t>(__popcll(same));
    pos[it] = c0 + static_cast<uint32_t>(__popcll(same & below));
  }
  __syncthreads();
  {
    const uint32_t d = tid;
    uint32_t c[W], tot = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      c[k] = wc[k][d];
      tot += c[k];
    }
    uint32_t all = 0;
    uint32_t run = block_exclusive_scan<kRsBlock>(tot, wsum, &all);
    tstart[d] = run;
    gofs[d] = offs[static_cast<uint64_t>(d) * n_tiles + blockIdx.x];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      wc[k][d] = run;
      run += c[k];
    }
  }
  __syncthreads();
  const uint32_t m = static_cast<uint32_t>(min(static_cast<uint64_t>(kRsTile), n - tile0));  // items of the tile
#pragma unroll
  for (int it = 0; it < kRsIter; ++it) {
    if (base + it * 64 + lane < n) {
      const uint32_t d = static_cast<uint32_t>(key[it] >> shift) & 255u;
      pos[it] += wc[w][d];
      stage[pos[it]] = key[it];
      sdig[pos[it]] = static_cast<uint8_t>(d);
    }
  }
  __syncthreads();
  for (uint32_t j = tid; j < m; j += kRsBlock) {
    const uint32_t d = sdig[j];
    keys_out[gofs[d] + (j - tstart[d])] = stage[j];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kRsIter; ++it) {
    const uint64_t i = base + it * 64 + lane;
    if (i < n) stage[pos[it]] = vals_in[i];
  }
  __syncthreads();
  for (uint32_t j = tid; j < m; j += kRsBlock) {
    const uint32_t d = sdig[j];
    vals_out[gofs[d] + (j - tstart[d])] = stage[j];
  }
}

// Every pair inside each run of equal keys: the thread at the run's first
// entry reports them.
__global__ __launch_bounds__(256) void k_a2_runs(const uint64_t* keys, const uint64_t* vals, uint64_t n, Cand* cand,
                                                uint32_t cand_cap, uint32_t* flags) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i + 1 < n; i += gridDim.x * 256ull) {
    const uint64_t k = keys[i];
    if (keys[i + 1] != k || (i > 0 && keys[i - 1] == k)) continue;
    uint64_t j = i + 1;
    while (j < n && keys[j] == k) ++j;
    for (uint64_t u = i; u < j; ++u)
      for (uint64_t v = u + 1; v < j; ++v) {
        const uint32_t slot = atomicAdd(&flags[kFlagCand], 1u);
        if (slot < cand_cap) {
          Cand c;
          c.a = make_entry(vals[u], k);
          c.b = make_entry(vals[v], k);
          cand[slot] = c;
        }
      }
  }
}

}  // namespace bx
