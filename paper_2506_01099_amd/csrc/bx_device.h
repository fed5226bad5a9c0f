// Device-side building blocks of the Benelux-pair search (gfx950).
//
// Layouts shared by the kernels:
//   Entry (12 B): one integer x that entered the join, as three 32-bit words
//     w0 = pos[0:32), w1 = pos[32:43) | fp[0:21) << 11, w2 = fp[21:53).
//   pos (43 bits) is x in single-range calls; in batched calls it is
//   x - a_query (28 bits) with the query index in bits 28..42.  fp (53 bits)
//   is a fingerprint of the set S_x = {rad(x), rad(x+1)} (and of the query in
//   batched calls): bits 11..63 of key64 of the canonical pair lo < hi.
//   Equal sets have equal fingerprints, so the join never misses a pair;
//   equal fingerprints of different sets are dropped by the verification,
//   which recomputes the four radicals by trial division.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bx {

constexpr uint32_t kGrpShift = 28;    // query id position inside pos (batched mode)
constexpr uint32_t kGrpMask = 0x7FFF;  // 15-bit query id in batched mode
constexpr uint32_t kFpBits = 53;

struct Entry {
  uint32_t w0, w1, w2;
};

// Odd prime power q = p^k (k >= 2) with its reciprocal (for q | x tests and the
// first-multiple offset) and p^{-1} mod 2^32 (for the exact division by p).
struct PrimePow {
  uint64_t q;
  double invq;
  uint32_t p;
  uint32_t pinv;
};

// Divisibility by an odd prime without division: p^-1 mod 2^64 and
// floor((2^64 - 1) / p) (zero for p = 2, which is tested by its low bit).
struct PrimeInv {
  uint64_t inv, lim;
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
constexpr int kDenseSlotMax = 2304;
// Slots a tile of T values needs at most (the odd prime powers q <= T with
// their floor(T/q) + 1 multiples: 555 for T = 2048, 2236 for T = 8192).
constexpr int dense_slot_cap(int T) { return T >= 8192 ? kDenseSlotMax : 576; }
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
  kFlagFalseCand = 6,  // equal fingerprints of different sets (dropped)
  kFlagWordMatch = 7,  // compact words with equal kept bits (each re-read from the first level)
  kFlagCount = 8
};

// 64-bit per-call counters (acc[]): entries written by the sieve, entries read
// by the join kernels (one add per partition).
enum : int { kAccEntries = 0, kAccJoined = 1, kAccCount = 2 };

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

// strip_two for x whose low 32-bit word is not zero (then ctz(x) is the
// count of the low word alone).
__device__ __forceinline__ uint64_t strip_two_lo(uint64_t x) {
  const uint32_t tz = static_cast<uint32_t>(__builtin_ctz(static_cast<uint32_t>(x)));
  return x >> (max(tz, 1u) - 1u);
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

// SplitMix64's output mix (Steele, Lea & Flood 2014): a bijection of 64-bit words.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// 64-bit hash of a join key: the canonical pair lo < hi (each below 2^43)
// and, in batched mode, the query id.  Bits 0..10 pick the first-level
// bucket, bits 11..63 are the entry's fingerprint (whose top bits pick the
// second-level partition and whose low bits the LDS table slot).  The word
// (lo | grp << 43) * K xor hi (K odd) is one-to-one in hi for a fixed lo,
// and two keys with different lo meet only if the top 21 bits of their
// products agree and the two hi differ by exactly the xor of the products;
// the SplitMix64 mix then spreads every bit (three 64-bit products in all).
__device__ __forceinline__ uint64_t key64(uint64_t lo, uint64_t hi, uint32_t grp) {
  return mix64(((lo | (static_cast<uint64_t>(grp) << 43)) * 0x9E3779B97F4A7C15ull) ^ hi);
}

__device__ __forceinline__ uint64_t entry_pos43(const Entry& e) {
  return e.w0 | (static_cast<uint64_t>(e.w1 & 0x7FFu) << 32);
}
__device__ __forceinline__ uint64_t entry_fp(const Entry& e) {
  return (e.w1 >> 11) | (static_cast<uint64_t>(e.w2) << 21);
}
__device__ __forceinline__ uint32_t entry_grp(const Entry& e, uint32_t gmask) {
  return static_cast<uint32_t>(entry_pos43(e) >> kGrpShift) & gmask;
}

// Position stored in an entry: plain mode x (43 bits), batched mode x - a (28 bits).
__device__ __forceinline__ uint64_t entry_pos(const Entry& e, int batch) {
  const uint64_t p = entry_pos43(e);
  return batch ? (p & ((1ull << kGrpShift) - 1)) : p;
}

// pos43 as described above; fp53 = key64(...) >> 11.
__device__ __forceinline__ Entry make_entry(uint64_t pos43, uint64_t fp53) {
  Entry e;
  e.w0 = static_cast<uint32_t>(pos43);
  e.w1 = static_cast<uint32_t>(pos43 >> 32) | (static_cast<uint32_t>(fp53) << 11);
  e.w2 = static_cast<uint32_t>(fp53 >> 21);
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
