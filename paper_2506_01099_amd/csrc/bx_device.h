// Device-side building blocks of the Benelux-pair search (gfx950).
//
// Layouts shared by the kernels:
//   Entry (16 B): the exact set S_x = {rad(x), rad(x+1)} of one integer x, with
//   the position of x, packed into two 64-bit words:
//     w0 = lo | (pos[0:22) << 42)
//     w1 = hi | (pos[22:..) << 42) | (grp << 48) | (orient << 63)
//   lo < hi are the two radicals (each below 2^42), orient = 1 when
//   rad(x) = hi.  Single-range calls store pos = x (43 bits, grp absent);
//   batched calls store pos = x - a_query (28 bits) and grp = query (15 bits).
//   The join key is (lo, hi) plus grp in batched mode.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bx {

constexpr uint64_t kM42 = (1ull << 42) - 1;
constexpr uint32_t kGrpShift = 48;
constexpr uint32_t kGrpMask = 0x7FFF;  // 15-bit query id in batched mode

struct Entry {
  uint64_t w0, w1;
};

// Odd prime power q = p^k (k >= 2) with its reciprocal (for q | x tests and the
// first-multiple offset) and p^{-1} mod 2^32 (for the exact division by p).
struct PrimePow {
  uint64_t q;
  double invq;
  uint32_t p;
  uint32_t pinv;
};

struct Query {
  uint64_t a, b;  // x in [a, b); radicals over [a, b]
};

struct Cand {
  Entry a, b;
};

struct OutPair {
  uint64_t m, n;
  uint32_t kind, query;
};

// Prime powers small enough to hit every LDS tile, with a static schedule that
// spreads their multiples over the threads of a workgroup: slot t belongs to
// power slot_d[t] and is its (t - prefix[d])-th multiple in the tile.
constexpr int kDenseMax = 64;
constexpr int kDenseSlotMax = 1152;
struct DenseTab {
  uint32_t n, nslots;
  uint32_t q[kDenseMax], p[kDenseMax], pinv[kDenseMax], prefix[kDenseMax];
  uint8_t slot_d[kDenseSlotMax];
};

// Indices into the per-call flag/counter words.
enum : int {
  kFlagL1Overflow = 0,
  kFlagL2Overflow = 1,
  kFlagCand = 2,
  kFlagOut = 3,
  kFlagVerifyFail = 4,
  kFlagSpillOverflow = 5,
  kFlagCount = 8
};

// Exact quotient r / p for an odd prime p dividing r, r < 2^64, from
// p^{-1} mod 2^32 (division by an invariant integer via its inverse,
// Granlund & Montgomery 1994).  With q = r / p = qh * 2^32 + ql:
// ql = r_lo * pinv (mod 2^32); r_hi = qh * p + mulhi(ql, p), so qh follows
// from the exact 32-bit division of r_hi - mulhi(ql, p) by p.
__device__ __forceinline__ uint64_t div_exact(uint64_t r, uint32_t p, uint32_t pinv) {
  const uint32_t ql = static_cast<uint32_t>(r) * pinv;
  const uint32_t t = static_cast<uint32_t>(r >> 32) - __umulhi(ql, p);
  const uint32_t qh = t * pinv;
  return (static_cast<uint64_t>(qh) << 32) | ql;
}

// p^{-1} mod 2^32 for odd p by Newton's iteration x <- x (2 - p x), which
// doubles the number of correct low bits; p itself is correct mod 2^3.
__device__ __forceinline__ uint32_t inv32(uint32_t p) {
  uint32_t x = p;
  x *= 2u - p * x;
  x *= 2u - p * x;
  x *= 2u - p * x;
  x *= 2u - p * x;
  return x;
}

// S mod q for S < 2^53 and 2 <= q < 2^53 with floor(S/q) < 2^31, from a
// double-precision quotient estimate that is off by at most one.
__device__ __forceinline__ uint64_t mod_fp64(uint64_t S, uint64_t q, double invq) {
  const double f = floor(static_cast<double>(S) * invq);
  int64_t r = static_cast<int64_t>(S) - static_cast<int64_t>(f) * static_cast<int64_t>(q);
  if (r < 0)
    r += static_cast<int64_t>(q);
  else if (r >= static_cast<int64_t>(q))
    r -= static_cast<int64_t>(q);
  return static_cast<uint64_t>(r);
}

// Divide the LDS cell by p (p divides it).  Different prime powers can hit the
// same cell at once, so the update is a 64-bit compare-and-swap loop.
__device__ __forceinline__ void lds_div(uint64_t* cell, uint32_t p, uint32_t pinv) {
  unsigned long long v = __atomic_load_n(reinterpret_cast<unsigned long long*>(cell), __ATOMIC_RELAXED);
  for (;;) {
    const unsigned long long nv = div_exact(v, p, pinv);
    const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(cell), v, nv);
    if (old == v) break;
    v = old;
  }
}

// rad(x) restricted to the prime 2: keep one factor 2 (shift by ctz(x) - 1
// when 4 | x), the count-trailing-zeros step of Section 3.1.
__device__ __forceinline__ uint64_t strip_two(uint64_t x) {
  const int tz = __builtin_ctzll(x);
  return tz >= 2 ? (x >> (tz - 1)) : x;
}

// u * v <= b for u, v, b < 2^43, without overflow.
__device__ __forceinline__ bool prod_le(uint64_t u, uint64_t v, uint64_t b) {
  return __umul64hi(u, v) == 0 && u * v <= b;
}

// Whether x can be a member of a pair (m, n) with m < n < b, given
// r0 = rad(x) and r1 = rad(x + 1).  Both kinds:
//  - the larger member n has n and n + 1 non-squarefree, except n = 3 in
//    (2, 3): a squarefree n or n + 1 would be the radical of a smaller number;
//  - if the smaller member m is squarefree, n or n + 1 equals m * t with
//    t >= 2, and every prime of m + 1 divides t - 1 (first kind) or t + 1
//    (second kind), so t >= max(2, rad(m + 1) - 1) and m * t <= b; the same
//    holds for m + 1 with rad(m), except t = 1, which forces (m, n) = (2, 3).
// So x is kept if x <= 3, or if every squarefree y of {x, x + 1} passes
// y * max(2, rad(other) - 1) <= b; x with both non-squarefree always passes.
__device__ __forceinline__ bool may_pair(uint64_t x, uint64_t r0, uint64_t r1, uint64_t b) {
  if (x <= 3) return true;
  if (r0 == x && !prod_le(x, r1 >= 3 ? r1 - 1 : 2, b)) return false;
  if (r1 == x + 1 && !prod_le(x + 1, r0 >= 3 ? r0 - 1 : 2, b)) return false;
  return true;
}

// Murmur3's 32-bit finalizer (Appleby): a bijective avalanche mix.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// Cheap hash of a join key, evaluated for every x to pick its pass: 21-bit
// limbs through full-rate 24-bit multiplies, then one xorshift-multiply round.
// Any function of the key gives exact passes; this one only has to spread the
// keys evenly.
__device__ __forceinline__ uint32_t pass_hash(uint64_t lo, uint64_t hi, uint32_t grp) {
  const uint32_t l0 = static_cast<uint32_t>(lo) & 0x1FFFFFu, l1 = static_cast<uint32_t>(lo >> 21);
  const uint32_t h0 = static_cast<uint32_t>(hi) & 0x1FFFFFu, h1 = static_cast<uint32_t>(hi >> 21);
  uint32_t s = __umul24(l0, 0x9E3779u) + __umul24(l1, 0x7F4A7Du) + __umul24(h0, 0xC2B2AFu) + __umul24(h1, 0x85EBCBu) +
               __umul24(grp, 0x27D4EBu);
  s ^= s >> 15;
  s *= 0x2C1B3C6Du;
  s ^= s >> 12;
  return s;
}

// Hash of a join key (lo, hi, grp) for the partition bits.  The key is
// canonical (lo < hi), so the hash is the same for both orders of the set.
__device__ __forceinline__ uint32_t key_hash(uint64_t lo, uint64_t hi, uint32_t grp) {
  const uint32_t c = (static_cast<uint32_t>(lo >> 32) | (static_cast<uint32_t>(hi >> 32) << 10)) + grp * 0x01000193u;
  return fmix32(static_cast<uint32_t>(lo) ^ fmix32(static_cast<uint32_t>(hi) ^ (c * 0x9E3779B1u)));
}

// An independent hash of the same key for the slots of the LDS join table.
__device__ __forceinline__ uint32_t key_hash2(uint64_t lo, uint64_t hi, uint32_t grp) {
  const uint32_t c = (static_cast<uint32_t>(lo >> 32) | (static_cast<uint32_t>(hi >> 32) << 10)) ^ (grp * 0x27D4EB2Fu);
  return fmix32(static_cast<uint32_t>(hi) ^ fmix32((static_cast<uint32_t>(lo) + 0x7F4A7C15u) ^ (c * 0x85EBCA77u)));
}

__device__ __forceinline__ uint64_t entry_lo(const Entry& e) { return e.w0 & kM42; }
__device__ __forceinline__ uint64_t entry_hi(const Entry& e) { return e.w1 & kM42; }
__device__ __forceinline__ uint32_t entry_grp(const Entry& e, uint32_t gmask) {
  return static_cast<uint32_t>(e.w1 >> kGrpShift) & gmask;
}

// Position stored in an entry: plain mode x (43 bits), batched mode x - a (28 bits).
__device__ __forceinline__ uint64_t entry_pos(const Entry& e, int batch) {
  const uint64_t low = e.w0 >> 42;
  const uint64_t high = (e.w1 >> 42) & (batch ? 0x3Full : 0x1FFFFFull);
  return low | (high << 22);
}

__device__ __forceinline__ Entry make_entry(uint64_t lo, uint64_t hi, uint64_t pos, uint32_t grp, uint32_t orient) {
  Entry e;
  e.w0 = lo | (pos << 42);
  e.w1 = hi | ((pos >> 22) << 42) | (static_cast<uint64_t>(grp) << kGrpShift) | (static_cast<uint64_t>(orient) << 63);
  return e;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Exclusive prefix sum over one value per thread of a workgroup of BLOCK
// threads; wsum holds BLOCK/64 words of scratch.  Returns the exclusive sum
// and writes the total to *total.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < NW ? wsum[lane] : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < NW) wsum[lane] = w;
  }
  __syncthreads();
  const uint32_t pre = wid ? wsum[wid - 1] : 0u;
  *total = wsum[NW - 1];
  return pre + x - v;
}

}  // namespace bx
