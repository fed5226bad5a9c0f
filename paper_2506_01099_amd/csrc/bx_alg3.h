// Algorithm 3 of the paper as a schedule of HIP kernels (the paper's own
// design, kept as a baseline beside the hash-partitioned passes).
//
// The search range is cut into chunks C_i of s integers that overlap by one
// (Section 2.2).  For chunk C_i the radicals are sieved (Algorithm 1, the
// radical sieve of this library), every n of the chunk but its last enters an
// open-addressing table of 4s slots in device memory (Section 3.1: a hash
// address in [0, 4s), four consecutive slots examined at once), and every
// equal key met on the way is a candidate pair (m, n) with both in C_i.  Then
// every earlier chunk C_j, j < i, is sieved again and each of its m probes the
// table up to the first empty slot: every equal key met is a candidate (m, n)
// with n in C_i.  Candidates go to the verification kernel, which recomputes
// the four radicals, so the table only needs a fingerprint of each set.
//
// A slot is one 64-bit word: the top 36 bits of the set's 64-bit key hash and
// the 28-bit index of n in its chunk; all ones marks an empty slot.  A word is
// claimed with one compare-and-swap, so an entry is never seen half written.
#pragma once
#include "bx_kernels.h"

namespace bx {

constexpr uint64_t kA3Empty = ~0ull;
constexpr int kA3IdxBits = 28;  // chunk index of n (chunks of at most 2^27 + 1 values)
constexpr uint64_t kA3IdxMask = (1ull << kA3IdxBits) - 1;
constexpr int kA3Probe = 4;     // slots examined at once

struct A3Params {
  const uint64_t* rad;  // rad[t] = rad(c0 + t), t in [0, count]
  uint64_t c0;          // first value of the chunk
  uint32_t count;       // entries of the chunk: c0 .. c0 + count - 1
  uint64_t* table;      // tmask + 1 slots
  uint64_t tmask;
  uint64_t n0;          // first value of the chunk whose entries the table holds (probe)
  Cand* cand;
  uint32_t cand_cap;
  uint32_t* flags;
};

__device__ __forceinline__ void a3_key(const A3Params& P, uint32_t t, uint64_t* fp, uint64_t* home) {
  const uint64_t a = P.rad[t], b = P.rad[t + 1];
  const uint64_t h = key64(a < b ? a : b, a < b ? b : a, 0);
  *fp = h;
  *home = (h >> 11) & P.tmask;  // hash address in [0, 4s)
}

__device__ __forceinline__ void a3_emit(const A3Params& P, uint64_t m, uint64_t n, uint64_t fp) {
  const uint32_t k = atomicAdd(&P.flags[kFlagCand], 1u);
  if (k < P.cand_cap) {
    Cand c;
    c.a = make_entry(m, fp >> 11);
    c.b = make_entry(n, fp >> 11);
    P.cand[k] = c;
  }
}

// Insert every n of the chunk (one thread per n, grid-stride).  Two equal keys
// walk the same probe sequence, so the one inserted later passes the other and
// reports the pair once.
__global__ __launch_bounds__(256) void k_a3_insert(A3Params P) {
  const uint64_t fpm = ~kA3IdxMask;
  for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < P.count; t += gridDim.x * 256ull) {
    uint64_t fp, s;
    a3_key(P, static_cast<uint32_t>(t), &fp, &s);
    const uint64_t mine = (fp & fpm) | t;
    bool placed = false;
    while (!placed) {
      uint64_t w[kA3Probe];
#pragma unroll
      for (int k = 0; k < kA3Probe; ++k) w[k] = __atomic_load_n(&P.table[(s + k) & P.tmask], __ATOMIC_RELAXED);
      int k = 0;
      for (; k < kA3Probe && !placed; ++k) {
        const uint64_t slot = (s + k) & P.tmask;
        uint64_t v = w[k];
        if (v == kA3Empty) {
          v = atomicCAS(reinterpret_cast<unsigned long long*>(&P.table[slot]), kA3Empty, mine);
          if (v == kA3Empty) {
            placed = true;
            break;
          }
        }
        // Occupied (possibly just now by another n): compare and walk on.
        if ((v & fpm) == (fp & fpm)) a3_emit(P, P.c0 + (v & kA3IdxMask), P.c0 + t, fp);
      }
      s = (s + k) & P.tmask;
    }
  }
}

// Probe the table (holding chunk C_i, first value n0) with every m of an earlier
// chunk, up to the first empty slot.
__global__ __launch_bounds__(256) void k_a3_probe(A3Params P) {
  const uint64_t fpm = ~kA3IdxMask;
  for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < P.count; t += gridDim.x * 256ull) {
    uint64_t fp, s;
    a3_key(P, static_cast<uint32_t>(t), &fp, &s);
    for (bool more = true; more;) {
      uint64_t w[kA3Probe];
#pragma unroll
      for (int k = 0; k < kA3Probe; ++k) w[k] = P.table[(s + k) & P.tmask];
#pragma unroll
      for (int k = 0; k < kA3Probe; ++k) {
        if (!more) break;
        if (w[k] == kA3Empty) {
          more = false;
        } else if ((w[k] & fpm) == (fp & fpm)) {
          a3_emit(P, P.c0 + t, P.n0 + (w[k] & kA3IdxMask), fp);
        }
      }
      s = (s + kA3Probe) & P.tmask;
    }
  }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

}  // namespace bx
