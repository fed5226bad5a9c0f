// Benelux-pair oracle: TEST INFRASTRUCTURE ONLY.
//
// A plain, slow CPU implementation of what the GPU path computes, used by the
// test-suite, by the smoke check and by the CPU-baseline leg of the benchmark
// to check the HIP library.  Nothing in the product library includes, links or
// calls this file, and this file shares no code with it.
//
// What is computed (Hercher, "On one of Erdos' Problems -- An Efficient Search
// for Benelux Pairs", arXiv:2506.01099):
//   * rad(n), the product of the distinct primes dividing n, with rad(1) = 1
//     (Section 2.1, definition of the radical).  Computed here by plain trial
//     division, the textbook definition, not by the paper's sieve (Algorithm 1).
//   * the set S_x = {rad(x), rad(x+1)} for every x of the range (Section 2.1,
//     the sets S_n built before Algorithm 2).
//   * every pair m < n with S_m = S_n.  It is of the first kind when
//     rad(m) = rad(n) (then also rad(m+1) = rad(n+1)) and of the second kind
//     otherwise (rad(m) = rad(n+1), rad(m+1) = rad(n)); Section 1 defines both
//     kinds and Algorithm 2 classifies a collision this way.
//   * ALL pairs inside a group of equal sets are reported, as the probe chains
//     of Algorithm 3 do (each insert/probe walks every occupied slot until an
//     empty one), and unlike the adjacent-only comparison printed in
//     Algorithm 2, which would skip the pair (2,8) of the group {2,3,8}.
//
//   * Erdos's original question (abstract and Section 1) adds a third
//     condition, rad(m+2) = rad(n+2).  With the kinds bit 4 a first-kind pair
//     that also meets rad(m+d) = rad(n+d) is reported with kind 5 (= 1 | 4);
//     d = 2 is the question as asked, other offsets d serve the tests (d = 1
//     repeats the second condition, so every first-kind pair meets it).  The
//     two radicals are taken by trial division, the definition.
//
// Ranges: a range query [a, b) reports pairs with max(a,1) <= m < n < b, so it
// needs radicals over [max(a,1), b].  search(N) is the range [1, N+1): pairs
// with n <= N.  Zero is not a positive integer and is never part of a range.
//
// Pins (tests/test_oracle.py): brute force by the definition over all
// m < n <= 2^12, the two infinite families and the two exceptional pairs of
// Section 1, Theorem 1's complete list, the paper's Tables 1 and 2, the count
// of squarefree integers via the Moebius function, and radical properties.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

// Trial division, definition of the radical (Section 2.1).
uint64_t rad_trial(uint64_t x) {
  if (x == 0) return 0;  // undefined; never asked for
  uint64_t r = 1;
  if ((x & 1) == 0) {
    r = 2;
    while ((x & 1) == 0) x >>= 1;
  }
  for (uint64_t d = 3; d <= x / d; d += 2) {
    if (x % d == 0) {
      r *= d;
      while (x % d == 0) x /= d;
    }
  }
  if (x > 1) r *= x;
  return r;
}

int pick_threads(int threads) {
  if (threads > 0) return threads;
  unsigned hc = std::thread::hardware_concurrency();
  return hc ? static_cast<int>(hc) : 1;
}

// rad(lo + i) for i in [0, hi - lo), static chunks over host threads.
void radicals_mt(uint64_t lo, uint64_t hi, uint64_t* out, int threads) {
  const uint64_t n = hi - lo;
  const int t = std::max(1, std::min<int>(pick_threads(threads), static_cast<int>(std::min<uint64_t>(n, 4096))));
  std::vector<std::thread> pool;
  for (int k = 0; k < t; ++k) {
    const uint64_t b = n * k / t, e = n * (k + 1) / t;
    pool.emplace_back([=] {
      for (uint64_t i = b; i < e; ++i) out[i] = rad_trial(lo + i);
    });
  }
  for (auto& th : pool) th.join();
}

struct KeyHash {
  size_t operator()(const std::pair<uint64_t, uint64_t>& k) const noexcept {
    return std::hash<uint64_t>()(k.first) ^ (std::hash<uint64_t>()(k.second) * 0x9E3779B97F4A7C15ull);
  }
};

}  // namespace

extern "C" {

// Pair record returned to the caller: (m, n, kind) with kind 1 or 2.
struct orc_pair {
  uint64_t m;
  uint64_t n;
  uint32_t kind;
  uint32_t reserved;
};

uint64_t orc_rad(uint64_t x) { return rad_trial(x); }

// out[i] = rad(lo + i) for i in [0, hi - lo); lo >= 1.  Returns 0, or -1 on bad args.
int orc_radicals(uint64_t lo, uint64_t hi, uint64_t* out, int threads) {
  if (lo == 0 || hi < lo || (hi > lo && out == nullptr)) return -1;
  if (hi == lo) return 0;
  radicals_mt(lo, hi, out, threads);
  return 0;
}

// All pairs max(a,1) <= m < n < b whose kind is in the mask `kinds`
// (1 = first, 2 = second, 4 = first kind and the third condition with offset
// third_offset, reported as kind 5; any mask in 1..7), sorted by (m, n).  A
// pair is reported when its kind (1 or 2) is in the mask, or when bit 4 is set
// and it is a first-kind pair with rad(m + d) = rad(n + d), d = third_offset;
// its kind is then 5.  *out is malloc'd and released with orc_free.  Timings
// of the two phases go to t_rad / t_join (seconds) when those pointers are
// non-null.  Returns 0, or -1 on bad args, -3 when memory runs out.
int orc_search_range_ex(uint64_t a, uint64_t b, uint32_t kinds, uint32_t third_offset, int threads, orc_pair** out,
                        size_t* count, double* t_rad, double* t_join) {
  if (!out || !count || kinds < 1 || kinds > 7) return -1;
  *out = nullptr;
  *count = 0;
  if (a == 0) a = 1;
  if (b <= a + 1) return 0;  // fewer than two integers: no pair
  // Radicals over [a, b]: S_x for x in [a, b) needs rad(x + 1) with x + 1 <= b.
  const uint64_t n_rad = b - a + 1;
  std::vector<uint64_t> r;
  try {
    r.resize(n_rad);
  } catch (...) {
    return -3;
  }
  auto c0 = std::chrono::steady_clock::now();
  radicals_mt(a, b + 1, r.data(), threads);
  auto c1 = std::chrono::steady_clock::now();

  // Group every x by its set S_x = {rad(x), rad(x+1)}, stored as (min, max).
  std::unordered_map<std::pair<uint64_t, uint64_t>, std::vector<uint64_t>, KeyHash> groups;
  std::vector<orc_pair> pairs;
  try {
    groups.reserve(static_cast<size_t>(b - a));
    for (uint64_t x = a; x < b; ++x) {
      const uint64_t u = r[x - a], v = r[x + 1 - a];
      groups[{std::min(u, v), std::max(u, v)}].push_back(x);
    }
    // Every pair inside every group; the kind compares rad(m) with rad(n).
    for (const auto& g : groups) {
      const std::vector<uint64_t>& xs = g.second;
      for (size_t i = 0; i < xs.size(); ++i)
        for (size_t j = i + 1; j < xs.size(); ++j) {
          const uint64_t m = std::min(xs[i], xs[j]), n = std::max(xs[i], xs[j]);
          const uint32_t kind = (r[m - a] == r[n - a]) ? 1u : 2u;
          // Third condition (Section 1): only a first-kind pair can meet all three.
          const bool third = (kinds & 4u) && kind == 1u &&
                             rad_trial(m + third_offset) == rad_trial(n + third_offset);
          if (third)
            pairs.push_back({m, n, kind | 4u, 0u});
          else if (kinds & kind)
            pairs.push_back({m, n, kind, 0u});
        }
    }
  } catch (...) {
    return -3;
  }
  std::sort(pairs.begin(), pairs.end(), [](const orc_pair& p, const orc_pair& q) {
    return p.m != q.m ? p.m < q.m : p.n < q.n;
  });
  auto c2 = std::chrono::steady_clock::now();
  if (t_rad) *t_rad = std::chrono::duration<double>(c1 - c0).count();
  if (t_join) *t_join = std::chrono::duration<double>(c2 - c1).count();

  if (!pairs.empty()) {
    orc_pair* p = static_cast<orc_pair*>(std::malloc(pairs.size() * sizeof(orc_pair)));
    if (!p) return -3;
    std::memcpy(p, pairs.data(), pairs.size() * sizeof(orc_pair));
    *out = p;
  }
  *count = pairs.size();
  return 0;
}

// The two kinds only (mask 1..3), as Algorithm 2 reports them.
int orc_search_range(uint64_t a, uint64_t b, uint32_t kinds, int threads, orc_pair** out, size_t* count,
                     double* t_rad, double* t_join) {
  if (kinds > 3) return -1;
  return orc_search_range_ex(a, b, kinds, 2, threads, out, count, t_rad, t_join);
}

void orc_free(void* p) { std::free(p); }

}  // extern "C"
