// Host side of the Benelux-pair search library: context, prime tables, the
// planner for the hash-partitioned passes, kernel orchestration and the C-ABI
// declared in include/benelux.h.
#include "benelux.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bx_alg2.h"
#include "bx_alg3.h"
#include "bx_kernels.h"
#include "bx_small.h"

using namespace bx;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define BX_HIP(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(BX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Two sieve shapes: LDS tiles of 2048 values with 512 threads (under 80 KB of
// LDS, two workgroups per CU) or 8192 values with 1024 threads (one per CU;
// eight values per thread between barriers, the faster shape).
constexpr int kTileSmall = 2048, kTileLarge = 8192;
constexpr int kTileDefault = kTileLarge;  // one 1024-thread workgroup per CU
constexpr int kVerifyGrid = 2048;
constexpr int kPartBlock = 1024;
constexpr int kJoinBlock = 1024;
constexpr int kVerifyBlock = 256;
constexpr uint32_t kCandCap = 1u << 20;
constexpr uint32_t kDefaultSegLen = 1u << 18;
constexpr uint64_t kMaxQueryLen = 1ull << 28;
constexpr uint32_t kMaxQueries = kGrpMask + 1;

enum { K_SIEVE = 0, K_PART = 1, K_JOIN = 2, K_VERIFY = 3, K_RAD = 4, K_SMALL = 5 };

// Queries of at most this many integers are served whole by one workgroup
// (k_small) when the small-query class is on; the class keeps no HBM entries.
constexpr uint32_t kSmallMaxLen = 8192;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t isqrt64(uint64_t n) {
  uint64_t r = static_cast<uint64_t>(std::sqrt(static_cast<double>(n)));
  while (r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}

uint32_t inv32_host(uint32_t p) {
  uint32_t x = p;
  for (int i = 0; i < 5; ++i) x *= 2u - p * x;
  return x;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Plan {
  uint32_t passes = 1, b1bits = 0, b2bits = 0, group = 1;
  uint64_t cap1 = 0;
  uint32_t cap2 = 0;
  uint64_t bytes = 0;
};

struct TimedLaunch {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct bx_ctx {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  uint64_t hi_max = 0, budget = 0;
  int n_cu = 256;
  std::string arch;
  std::vector<uint32_t> primes;
  std::vector<PrimePow> pp;
  std::vector<double> cum_inv_q;  // cum_inv_q[i] = sum of 1/q over pp[0, i)
  uint32_t n_dense[2] = {0, 0};  // per tile shape (small, large)
  uint32_t* d_primes = nullptr;
  PrimeInv* d_pinv = nullptr;  // per prime: p^-1 mod 2^64 and floor((2^64 - 1) / p) (divisibility tests)
  PrimePow* d_pp = nullptr;
  DenseTab* d_dense[2] = {nullptr, nullptr};
  DevBuf l1, l2, cnt1, cnt2, cand, out, flags, spill, queries, segpref, rad, acc, a3tab, smallq;
  DevBuf a2k[2], a2v[2], a2hist, a2offs, a2tot;  // Algorithm 2: list (double-buffered), sort counts
  int force_passes = 0, timing = 1, force_b1 = -1, force_b2 = -1, force_group = 0;
  int prune = 1;            // drop x that cannot be a pair member before the join
  int join_sort = 0;        // 1: the sort join per partition (ablation of the hash join)
  uint32_t third_off = 2;   // offset d of the third condition rad(m + d) = rad(n + d); 2 is Erdős's
  int schedule = 0;         // 0: hash-partitioned passes, 1: Algorithm 3's chunk schedule, 2: Algorithm 2's sort (baselines)
  uint32_t a3_log2 = 27;    // Algorithm 3's chunk size s = 2^a3_log2 (a table of 4s slots)
  // Fingerprint bits kept: all 53 in use; tests keep the top 11 (the
  // partition bits) and a few low ones to make different sets collide.
  uint64_t fp_mask = (1ull << kFpBits) - 1;
  int tile = kTileDefault;
  uint32_t small_max = kSmallMaxLen;  // longest query of the small class (0: class off)
  int small_block = 1024;             // threads of a small-class workgroup
  int submit_wait = 1;                // 0: bx_submit refuses what cannot be admitted at once
  int compact = 1;                    // 8-byte second-level words where the plan allows (0 = never)
  uint32_t compact_fp_bits = 0;       // tests: fingerprint bits a compact word keeps (0 = all it can)
  int graph_batch = 1;      // batched calls run as one captured HIP graph
  bool capturing = false;   // no event records while a stream capture is open
  hipGraphExec_t graph_exec = nullptr;
  std::string graph_key;
  uint32_t graph_launches[6] = {0, 0, 0, 0, 0, 0};  // kernel launches the graph holds, per kernel
  uint32_t seg_len = kDefaultSegLen;
  bx_stats stats{};
  std::mutex mu;
  std::vector<hipEvent_t> ev_free;
  std::vector<TimedLaunch> timed;
  hipEvent_t last_done = nullptr;    // recorded after the last call's work
  hipStream_t last_stream = nullptr;  // stream that work ran on
  void* na = nullptr;  // this device's no-allocation scratch (NaDevice)
  // Pinned host staging of the query tables (uploads need no wait for the host
  // vectors) and the event after their last upload (the next upload waits for it).
  void* pin = nullptr;
  size_t pin_bytes = 0;
  hipEvent_t pin_ev = nullptr;
  // serving
  struct Server;
  std::unique_ptr<Server> server;
};

namespace {

int ensure(bx_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return BX_OK;
  if (b.p) {
    BX_HIP(hipStreamSynchronize(c->stream));
    BX_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(BX_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return BX_OK;
}

void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

hipEvent_t get_event(bx_ctx* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct LaunchTimer {
  bx_ctx* c;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  LaunchTimer(bx_ctx* ctx, int k, hipStream_t st) : c(ctx), kind(k), s(st) {
    c->stats.launches[k]++;
    if (c->timing && !c->capturing) {
      a = get_event(c);
      b = get_event(c);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~LaunchTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      c->timed.push_back({kind, a, b});
    }
  }
};

// Called after the stream has drained: fold the recorded launches into stats.
void collect_timings(bx_ctx* c) {
  for (auto& t : c->timed) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) c->stats.kernel_ms[t.kind] += ms;
    c->ev_free.push_back(t.a);
    c->ev_free.push_back(t.b);
  }
  c->timed.clear();
}

void reset_stats(bx_ctx* c) {
  for (auto& t : c->timed) {
    c->ev_free.push_back(t.a);
    c->ev_free.push_back(t.b);
  }
  c->timed.clear();
  c->stats = bx_stats{};
}

// The workspace is shared by all calls of a context: work queued on a new
// stream first waits for the previous call's work on the old one.
int order_after_last(bx_ctx* c, hipStream_t st) {
  if (c->last_done && c->last_stream != st) BX_HIP(hipStreamWaitEvent(st, c->last_done, 0));
  return BX_OK;
}

int mark_done(bx_ctx* c, hipStream_t st) {
  if (!c->last_done) BX_HIP(hipEventCreateWithFlags(&c->last_done, hipEventDisableTiming));
  BX_HIP(hipEventRecord(c->last_done, st));
  c->last_stream = st;
  return BX_OK;
}

int fill_u32(bx_ctx* c, void* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return BX_OK;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, static_cast<uint32_t*>(p), n, v);
  BX_HIP(hipGetLastError());
  return BX_OK;
}

// Prime tables: primes <= isqrt(hi_max) (for verification) and every odd prime
// power p^k <= hi_max, k >= 2 (Algorithm 1 sieves with exactly these), sorted
// by q, plus the dense schedules for the powers <= each tile size.
int build_tables(bx_ctx* c) {
  const uint64_t lim = isqrt64(c->hi_max);
  std::vector<uint8_t> comp(lim + 1, 0);
  c->primes.clear();
  for (uint64_t i = 2; i <= lim; ++i) {
    if (comp[i]) continue;
    c->primes.push_back(static_cast<uint32_t>(i));
    for (uint64_t j = i * i; j <= lim; j += i) comp[j] = 1;
  }
  c->pp.clear();
  for (uint32_t p : c->primes) {
    if (p == 2) continue;
    const uint32_t pinv = inv32_host(p);
    uint64_t q = static_cast<uint64_t>(p) * p;
    while (q <= c->hi_max) {
      c->pp.push_back(PrimePow{q, 1.0 / static_cast<double>(q), p, pinv});
      if (q > c->hi_max / p) break;
      q *= p;
    }
  }
  std::sort(c->pp.begin(), c->pp.end(), [](const PrimePow& a, const PrimePow& b) { return a.q < b.q; });
  c->cum_inv_q.assign(c->pp.size() + 1, 0.0);
  for (size_t i = 0; i < c->pp.size(); ++i) c->cum_inv_q[i + 1] = c->cum_inv_q[i] + c->pp[i].invq;
  for (int which = 0; which < 2; ++which) {
    const uint32_t T = which ? kTileLarge : kTileSmall;
    DenseTab dt;
    std::memset(&dt, 0, sizeof(dt));
    uint32_t nd = 0, slots = 0;
    for (const auto& w : c->pp) {
      if (w.q > T) break;
      if (nd >= static_cast<uint32_t>(kDenseMax)) return fail(BX_EINTERNAL, "dense prime-power table overflow");
      const uint32_t q = static_cast<uint32_t>(w.q);
      const uint32_t ub = T / q + 1;  // multiples of q among T + 1 consecutive values
      if (slots + ub > static_cast<uint32_t>(dense_slot_cap(static_cast<int>(T))))
        return fail(BX_EINTERNAL, "dense slot table overflow");
      dt.q[nd] = q;
      dt.p[nd] = w.p;
      dt.pinv[nd] = w.pinv;
      dt.prefix[nd] = slots;
      for (uint32_t k = 0; k < ub; ++k) dt.slot_d[slots + k] = static_cast<uint8_t>(nd);
      slots += ub;
      ++nd;
    }
    dt.n = nd;
    dt.nslots = slots;
    c->n_dense[which] = nd;
    BX_HIP(hipMalloc(&c->d_dense[which], sizeof(DenseTab)));
    BX_HIP(hipMemcpy(c->d_dense[which], &dt, sizeof(DenseTab), hipMemcpyHostToDevice));
  }
  BX_HIP(hipMalloc(&c->d_primes, std::max<size_t>(4, c->primes.size() * sizeof(uint32_t))));
  {
    // x is a multiple of odd p iff x * p^-1 mod 2^64 <= floor((2^64 - 1) / p)
    // (Granlund & Montgomery 1994), and the product is then x / p.
    std::vector<PrimeInv> inv(c->primes.size());
    for (size_t i = 0; i < c->primes.size(); ++i) {
      const uint64_t p = c->primes[i];
      uint64_t x = p;  // p^-1 mod 2^3 for odd p; each Newton step doubles the correct bits
      for (int k = 0; k < 5; ++k) x *= 2 - p * x;
      inv[i] = PrimeInv{p & 1 ? x : 0, p & 1 ? UINT64_MAX / p : 0};
    }
    BX_HIP(hipMalloc(&c->d_pinv, std::max<size_t>(sizeof(PrimeInv), inv.size() * sizeof(PrimeInv))));
    if (!inv.empty())
      BX_HIP(hipMemcpy(c->d_pinv, inv.data(), inv.size() * sizeof(PrimeInv), hipMemcpyHostToDevice));
  }
  BX_HIP(hipMalloc(&c->d_pp, std::max<size_t>(sizeof(PrimePow), c->pp.size() * sizeof(PrimePow))));
  if (!c->primes.empty())
    BX_HIP(hipMemcpy(c->d_primes, c->primes.data(), c->primes.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  if (!c->pp.empty())
    BX_HIP(hipMemcpy(c->d_pp, c->pp.data(), c->pp.size() * sizeof(PrimePow), hipMemcpyHostToDevice));
  return BX_OK;
}

uint32_t ceil_log2(double v) {
  uint32_t b = 0;
  while (std::ldexp(1.0, static_cast<int>(b)) < v) ++b;
  return b;
}

uint64_t round_up(uint64_t v, uint64_t m) { return (v + m - 1) / m * m; }

// Sparse hits per workgroup beyond the sieve's LDS list (worst case).
uint32_t spill_cap_of(const bx_ctx* c) {
  return static_cast<uint32_t>(c->pp.size() - c->n_dense[0] + c->seg_len / 128 + 64);
}

uint64_t fixed_bytes(const bx_ctx* c, uint32_t sieve_grid) {
  return static_cast<uint64_t>(sieve_grid) * spill_cap_of(c) * 8ull + kCandCap * (sizeof(Cand) + sizeof(OutPair)) +
         (64ull << 20);
}

// Choose the number of hash passes P (any integer: pass p keeps the keys whose
// pass hash falls in the p-th of P equal ranges) and the two partition
// fan-outs.  One pass's entries live in the first-level buckets (12 B each);
// the second level only needs a buffer for one group of buckets at a time, so
// the budget sets P through the first level alone.  Second-level partitions
// end up near 3800-7600 entries, which one workgroup joins in LDS.
int make_plan(bx_ctx* c, uint64_t n_keys, uint64_t n_expect, uint64_t share, uint32_t sieve_grid, Plan* out) {
  const uint64_t fixed = fixed_bytes(c, sieve_grid);
  const uint32_t p_first = c->force_passes > 0 ? static_cast<uint32_t>(c->force_passes) : 1;
  const uint32_t p_last = c->force_passes > 0 ? p_first : 4096;
  const double W = static_cast<double>(sieve_grid);
  for (uint32_t P = p_first; P <= p_last; ++P) {
    Plan p;
    p.passes = P;
    // Fan-outs from the expected entries per pass; the regions from the bound.
    // The first level takes the fewest buckets whose second level still needs
    // at most 2^11 partitions: every partition and join launch then moves as
    // much as it can (a small search runs one of each instead of one per
    // group of a few thousand entries), and the sieve's flushes write longer
    // runs per bucket.
    const double n_pass = std::max(1.0, std::ceil(static_cast<double>(std::min(n_expect, n_keys)) / P));
    uint32_t b1 = std::min<uint32_t>(10, ceil_log2(n_pass * 1.03 / (7600.0 * 2048.0)));
    if (c->force_b1 >= 0) b1 = static_cast<uint32_t>(c->force_b1);
    p.b1bits = b1;
    const double bucket = n_pass / std::ldexp(1.0, static_cast<int>(b1));
    // Each sieve workgroup owns one region per bucket (no atomics); it holds
    // that workgroup's integers of the bucket and pass, plus slack.
    const double region = static_cast<double>(share) / P / std::ldexp(1.0, static_cast<int>(b1));
    p.cap1 = round_up(static_cast<uint64_t>(std::ceil(region * 1.05)) + 256, 64);
    (void)W;
    // Partitions of at most ~7.6k entries on average: with the bucket-to-bucket
    // spread (3%) and the partition-to-partition spread (a few sigma of ~90)
    // they stay within one LDS join chunk (8192 entries).
    uint32_t b2 = bucket * 1.03 > 7600.0 ? ceil_log2(bucket * 1.03 / 7600.0) : 0;
    if (c->force_b2 >= 0) b2 = static_cast<uint32_t>(c->force_b2);
    if (b2 > 11 || b1 + b2 > 32) {
      if (c->force_passes > 0) return fail(BX_ENOMEM, "forced pass count leaves partitions too large");
      continue;
    }
    p.b2bits = b2;
    p.cap2 = static_cast<uint32_t>(
        round_up(static_cast<uint64_t>(std::ceil(bucket * 1.03 / std::ldexp(1.0, static_cast<int>(b2)) * 1.1)) + 128, 16));
    if (p.cap1 > 0xF0000000ull || p.cap2 > 0xF0000000ull) continue;
    const uint64_t nb1 = 1ull << b1, nb2 = 1ull << b2;
    uint32_t G = c->force_group > 0 ? static_cast<uint32_t>(c->force_group) : 8u;
    if (G > nb1) G = static_cast<uint32_t>(nb1);
    p.group = G;
    p.bytes = nb1 * sieve_grid * p.cap1 * sizeof(Entry) + G * nb2 * p.cap2 * sizeof(Entry) +
              (nb1 * sieve_grid + G * nb2) * 4;
    if (p.bytes + fixed <= c->budget) {
      *out = p;
      return BX_OK;
    }
    if (c->force_passes > 0)
      return fail(BX_ENOMEM, "forced pass count needs " + std::to_string(p.bytes + fixed) + " bytes, budget " +
                                 std::to_string(c->budget));
  }
  return fail(BX_ENOMEM, "HBM budget too small for the search");
}

struct Segs {
  std::vector<Query> q;
  std::vector<uint64_t> prefix;
  std::vector<uint32_t> small;  // queries served by the small-query class (no segments)
  uint64_t n_segs = 0;
  uint64_t n_ints = 0;  // integers sieved
  uint64_t n_keys = 0;    // bound on the entries they produce (all of them without the member test)
  uint64_t n_expect = 0;  // expected entries
};

// Bounds on the entries the member test (may_pair) keeps in a query [a, b):
//  - x with x and x + 1 non-squarefree: density 0.1068, at most 0.122 in any
//    window of 2^10 integers (0.1077 in windows of 2^15); charged at 0.125;
//  - the other kept x lie at or below b / 2: all x <= 2 sqrt(b) may pass
//    (charged at 1), and above that only x + 1 or x with a small radical
//    pass: 1.1-1.2 sqrt(b) of them for b from 2^20 to 2^26, charged as
//    2 sqrt(b) per query.
// A region that still overflows is caught and its pass split, so these
// bounds affect speed only.
constexpr int kZones = 2;
constexpr double kZoneRate[kZones] = {1.0, 0.125};

double sqrt_b(const Query& q) { return std::sqrt(static_cast<double>(q.b)); }

// Zone k of query q covers x in [zone_lo(k), zone_lo(k + 1)).
uint64_t zone_lo(const Query& q, int k) {
  if (k == 0) return 0;
  if (k == kZones) return UINT64_MAX;
  return static_cast<uint64_t>(2.0 * sqrt_b(q)) + 4;
}

// The scattered kept x above 2 sqrt(b) (none when the query lies above b / 2).
double scattered(const bx_ctx* c, const Query& q) {
  if (!c->prune || q.a > q.b / 2) return 0.0;
  return 2.0 * sqrt_b(q);
}

double rate_at(const bx_ctx* c, const Query& q, uint64_t x) {
  if (!c->prune) return 1.0;
  int k = 0;
  while (k + 1 < kZones && x >= zone_lo(q, k + 1)) ++k;
  return kZoneRate[k];
}

// Expected number of kept x in query q: the both-non-squarefree density
// (0.1068, at most 0.1077 in any window of 2^15), the low zone and ~1.2 sqrt(b)
// scattered ones.
double kept_expected(const bx_ctx* c, const Query& q) {
  if (q.b <= q.a) return 0.0;
  if (!c->prune) return static_cast<double>(q.b - q.a);
  const uint64_t low = std::min(q.b, std::max(q.a, zone_lo(q, 1)));
  return static_cast<double>(low - q.a) + 0.108 * static_cast<double>(q.b - low) +
         (q.a > q.b / 2 ? 0.0 : 1.2 * sqrt_b(q)) + 3.0;
}

// Bound on the number of kept x in [u, v) of query q.
double kept_bound(const bx_ctx* c, const Query& q, uint64_t u, uint64_t v) {
  if (v <= u) return 0.0;
  if (!c->prune) return static_cast<double>(v - u);
  double n = 0.0;
  for (int k = 0; k < kZones; ++k) {
    const uint64_t l = std::max(u, zone_lo(q, k)), h = std::min(v, zone_lo(q, k + 1));
    if (h > l) n += kZoneRate[k] * static_cast<double>(h - l);
  }
  return n + scattered(c, q) + 3.0;  // x <= 3
}

// Adds w to every workgroup that runs one of the segments [g, g + n) (segment
// s runs on workgroup s mod W), through a difference array.
void add_round_robin(std::vector<double>& diff, uint64_t g, uint64_t n, uint32_t W, double w) {
  if (n == 0 || w == 0.0) return;
  const double rounds = static_cast<double>(n / W);
  const uint64_t rem = n % W, first = g % W;
  diff[0] += rounds * w;
  diff[W] -= rounds * w;
  if (rem) {
    const uint64_t end = first + rem;  // [first, end) mod W get one more
    if (end <= W) {
      diff[first] += w;
      diff[end] -= w;
    } else {
      diff[first] += w;
      diff[W] -= w;
      diff[0] += w;
      diff[end - W] -= w;
    }
  }
}

// The largest number of kept x that one sieve workgroup can produce (an upper
// bound).  Segments run round-robin; a segment is charged at the rate of the
// zone holding its first integer, the highest rate it touches.
uint64_t max_share(const bx_ctx* c, const Segs& s, uint32_t W) {
  if (W == 0) return 0;
  std::vector<double> diff(W + 1, 0.0);
  std::vector<double> extra(W, 0.0);  // the shorter last segment of each query
  const uint64_t L = c->seg_len;
  for (size_t i = 0; i < s.q.size(); ++i) {
    const Query& q = s.q[i];
    const uint64_t len = q.b > q.a ? q.b - q.a : 0;
    if (len == 0 || s.prefix[i + 1] == s.prefix[i]) continue;  // empty or small-class
    const uint64_t nseg = (len + L - 1) / L, nfull = nseg - 1;
    // Full segments, split where the zone changes.
    uint64_t k = 0;
    while (k < nfull) {
      const uint64_t x = q.a + k * L;
      const double r = rate_at(c, q, x);
      uint64_t k_end = nfull;
      if (c->prune)
        for (int z = 1; z < kZones; ++z) {
          const uint64_t zl = zone_lo(q, z);
          if (zl > x) {  // first segment whose start lies at or past zl
            k_end = std::min(nfull, (zl - q.a + L - 1) / L);
            break;
          }
        }
      if (k_end <= k) k_end = k + 1;
      add_round_robin(diff, s.prefix[i] + k, k_end - k, W, r * static_cast<double>(L));
      k = k_end;
    }
    const uint64_t x_last = q.a + nfull * L;
    extra[(s.prefix[i] + nfull) % W] += rate_at(c, q, x_last) * static_cast<double>(len - nfull * L) + 3.0;
  }
  // The scattered kept x of each query, charged to every workgroup at four
  // times an even spread over the query's segments.
  double spread = 0.0;
  for (size_t i = 0; i < s.q.size(); ++i) {
    const uint64_t nseg = s.prefix[i + 1] - s.prefix[i];
    if (nseg == 0) continue;
    const double sc = scattered(c, s.q[i]);
    if (sc == 0.0) continue;
    const double per = 4.0 * sc * static_cast<double>((nseg + W - 1) / W) / static_cast<double>(std::max<uint64_t>(1, nseg));
    spread += std::min(sc, per) + 64.0;
  }
  double best = 0.0, run = 0.0;
  for (uint32_t w = 0; w < W; ++w) {
    run += diff[w];
    best = std::max(best, run + extra[w]);
  }
  return static_cast<uint64_t>(std::ceil(best + spread));
}

// Whether query q is served by the small-query class.
bool is_small(const bx_ctx* c, const Query& q) {
  const uint64_t L = q.b > q.a ? q.b - q.a : 0;
  return L >= 2 && L <= c->small_max;
}

// Segments of every query; with small_class, the queries of the small-query
// class take none and are listed in s->small instead (searches only: the
// radical sieve segments every range).
void make_segs(const bx_ctx* c, Segs* s, bool small_class) {
  s->prefix.assign(s->q.size() + 1, 0);
  s->small.clear();
  s->n_ints = 0;
  uint64_t acc = 0;
  double keys = 0.0, expect = 0.0;
  for (size_t i = 0; i < s->q.size(); ++i) {
    s->prefix[i] = acc;
    const uint64_t L = s->q[i].b > s->q[i].a ? s->q[i].b - s->q[i].a : 0;
    if (small_class && is_small(c, s->q[i])) {
      s->small.push_back(static_cast<uint32_t>(i));
      s->n_ints += L;
      continue;
    }
    acc += (L + c->seg_len - 1) / c->seg_len;
    keys += kept_bound(c, s->q[i], s->q[i].a, s->q[i].b);
    expect += kept_expected(c, s->q[i]);
    s->n_ints += L;
  }
  s->prefix[s->q.size()] = acc;
  s->n_segs = acc;
  s->n_keys = static_cast<uint64_t>(std::ceil(keys));
  s->n_expect = static_cast<uint64_t>(std::ceil(expect));
}

// Uploads the query table, the segment prefix and the small-query list through
// the context's pinned staging buffer: the copies are queued on st and the
// call returns at once (the next upload waits for these copies first).  The
// device tables are rewritten only once the kernels queued before on st,
// which may read them, have finished: a small copy from pinned memory may be
// carried out by the host at once rather than in stream order.
int upload_segs(bx_ctx* c, const Segs& s, hipStream_t st) {
  int rc;
  if ((rc = ensure(c, c->queries, s.q.size() * sizeof(Query))) != BX_OK) return rc;
  if ((rc = ensure(c, c->segpref, s.prefix.size() * sizeof(uint64_t))) != BX_OK) return rc;
  if (!s.small.empty() && (rc = ensure(c, c->smallq, s.small.size() * sizeof(uint32_t))) != BX_OK) return rc;
  const size_t nq = s.q.size() * sizeof(Query), np = s.prefix.size() * sizeof(uint64_t),
               ns = s.small.size() * sizeof(uint32_t);
  const size_t op = (nq + 63) & ~size_t(63), os = op + ((np + 63) & ~size_t(63)), need = os + ns;
  if (c->pin_ev) BX_HIP(hipEventSynchronize(c->pin_ev));  // the previous upload has left the buffer
  BX_HIP(hipStreamSynchronize(st));  // earlier kernels are done with the tables
  if (need > c->pin_bytes) {
    if (c->pin) BX_HIP(hipHostFree(c->pin));
    c->pin = nullptr;
    c->pin_bytes = 0;
    const size_t bytes = std::max<size_t>(need, 1 << 16);
    if (hipHostMalloc(&c->pin, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c->pin = nullptr;
      return fail(BX_ENOMEM, "pinned host allocation of " + std::to_string(bytes) + " bytes failed");
    }
    c->pin_bytes = bytes;
  }
  if (!c->pin_ev) BX_HIP(hipEventCreateWithFlags(&c->pin_ev, hipEventDisableTiming));
  uint8_t* h = static_cast<uint8_t*>(c->pin);
  std::memcpy(h, s.q.data(), nq);
  std::memcpy(h + op, s.prefix.data(), np);
  if (ns) std::memcpy(h + os, s.small.data(), ns);
  BX_HIP(hipMemcpyAsync(c->queries.p, h, nq, hipMemcpyHostToDevice, st));
  BX_HIP(hipMemcpyAsync(c->segpref.p, h + op, np, hipMemcpyHostToDevice, st));
  if (ns) BX_HIP(hipMemcpyAsync(c->smallq.p, h + os, ns, hipMemcpyHostToDevice, st));
  if (!c->capturing) BX_HIP(hipEventRecord(c->pin_ev, st));
  return BX_OK;
}

SieveParams base_sieve_params(bx_ctx* c, const Segs& s) {
  SieveParams P;
  std::memset(&P, 0, sizeof(P));
  P.queries = static_cast<const Query*>(c->queries.p);
  P.seg_prefix = static_cast<const uint64_t*>(c->segpref.p);
  P.n_queries = static_cast<uint32_t>(s.q.size());
  P.n_segs = s.n_segs;
  P.seg_len = c->seg_len;
  P.pp = c->d_pp;
  P.n_pp = static_cast<uint32_t>(c->pp.size());
  const int which = c->tile == kTileLarge ? 1 : 0;
  P.n_dense = c->n_dense[which];
  P.dense = c->d_dense[which];
  P.spill = static_cast<uint64_t*>(c->spill.p);
  P.spill_cap = spill_cap_of(c);
  P.flags = static_cast<uint32_t*>(c->flags.p);
  return P;
}

int check_query(const bx_ctx* c, uint64_t a, uint64_t b, uint32_t kinds) {
  // The third condition takes rad(n + d), n <= b - 1, by trial division.
  const uint64_t top = (kinds & BX_THIRD) ? std::max<uint64_t>(b, b - 1 + c->third_off) : b;
  if (top > c->hi_max || top >= BX_VALUE_LIMIT)
    return fail(BX_ERANGE, "range end " + std::to_string(b) + " exceeds hi_max " + std::to_string(c->hi_max));
  (void)a;
  return BX_OK;
}

template <int MODE>
void launch_sieve(const bx_ctx* c, const SieveParams& P, uint32_t grid, hipStream_t st) {
  if (c->tile == kTileLarge)
    hipLaunchKernelGGL((k_sieve<kTileLarge, 1024, MODE>), dim3(grid), dim3(1024), 0, st, P);
  else
    hipLaunchKernelGGL((k_sieve<kTileSmall, 512, MODE>), dim3(grid), dim3(512), 0, st, P);
}

// Sieve workgroups per CU for the key-generating sieve (LDS bound).
uint32_t sieve_wg_per_cu(const bx_ctx* c) { return c->tile == kTileLarge ? 1u : 2u; }

// One search: plan, buffers and launch shapes.
struct Job {
  Segs* s = nullptr;
  int batch = 0;
  uint32_t kinds = 3;
  Plan plan;
  uint32_t sieve_grid = 0, B1 = 1, B2 = 1, G = 1, cpr = 1;
  uint64_t ngsub = 1, n_regions = 1, part_grid = 8;
  uint32_t gmask = 0;
  // Compact second level (8-byte words): the entry's index among its bucket's
  // first-level regions, the low fingerprint bits above it.
  bool compact = false;
  uint32_t idx_bits = 0;
  uint64_t low_mask = 0;
};

// Random matches of kept word bits a compact plan expects (pairs of different
// sets whose kept fingerprint bits, bucket and partition agree; the join reads
// both entries of each back from the first level), at most this many per call.
constexpr double kCompactMatchMax = 3e5;

// Bytes of every workspace buffer a job needs.
struct JobBufs {
  size_t l1, l2, cnt1, cnt2, cand, out, flags, acc, spill, queries, segpref, smallq;
};

// The plan and launch shapes of one search over `s` and the workspace it
// needs; nothing is allocated.
int plan_job(bx_ctx* c, Segs& s, int batch, uint32_t kinds, Job* j, JobBufs* nb) {
  int rc;
  j->s = &s;
  j->batch = batch;
  j->kinds = kinds;
  j->sieve_grid =
      static_cast<uint32_t>(std::min<uint64_t>(s.n_segs, static_cast<uint64_t>(c->n_cu) * sieve_wg_per_cu(c)));
  if ((rc = make_plan(c, s.n_keys, s.n_expect, max_share(c, s, j->sieve_grid), j->sieve_grid, &j->plan)) != BX_OK)
    return rc;
  const Plan& plan = j->plan;
  j->B1 = 1u << plan.b1bits;
  j->B2 = 1u << plan.b2bits;
  j->G = plan.group;
  j->ngsub = static_cast<uint64_t>(j->G) * j->B2;
  j->n_regions = static_cast<uint64_t>(j->B1) * j->sieve_grid;
  j->cpr = static_cast<uint32_t>((plan.cap1 + kPartChunk - 1) / kPartChunk);
  const uint64_t chunks = static_cast<uint64_t>(j->sieve_grid) * j->cpr;  // per bucket
  // Persistent partition grid: one workgroup per CU (measured faster than two), a multiple
  // of 8 so that every XCD serves its share of the group's buckets.
  const uint64_t per = 8 / j->G;
  j->part_grid = 8ull * std::min<uint64_t>(std::max(1, c->n_cu / 8), (chunks + per - 1) / per);
  if (j->part_grid > 0x7FFFFFFFull) return fail(BX_EINTERNAL, "partition grid too large");
  j->gmask = batch ? kGrpMask : 0u;
  nb->l1 = j->n_regions * plan.cap1 * sizeof(Entry);
  // Compact words need the full fingerprint (no test mask), the hash join, and
  // enough kept bits that random matches stay few.
  {
    const uint64_t per_bucket = static_cast<uint64_t>(j->sieve_grid) * plan.cap1;  // first-level slots of a bucket
    uint32_t ib = 1;
    while (ib < 64 && (1ull << ib) < per_bucket) ++ib;
    j->idx_bits = ib;
    const uint32_t f2 = std::min<uint32_t>(kFpBits, 64 - ib);
    const uint32_t keep = c->compact_fp_bits ? std::min(f2, c->compact_fp_bits) : f2;
    const double per_pass = static_cast<double>(s.n_expect) / plan.passes;
    const double match_est =
        plan.passes * per_pass * per_pass / 2.0 / std::ldexp(1.0, static_cast<int>(keep + plan.b1bits + plan.b2bits));
    j->compact = c->compact && c->fp_mask == (1ull << kFpBits) - 1 && !c->join_sort && f2 >= 24 &&
                 (c->compact_fp_bits || match_est <= kCompactMatchMax);
    if (j->compact) j->low_mask = (1ull << keep) - 1;
  }
  nb->l2 = j->ngsub * plan.cap2 * (j->compact ? sizeof(uint64_t) : sizeof(Entry));
  nb->cnt1 = j->n_regions * 4ull;
  nb->cnt2 = j->ngsub * 4ull;
  nb->cand = kCandCap * sizeof(Cand);
  nb->out = kCandCap * sizeof(OutPair);
  nb->flags = kFlagCount * 4;
  nb->acc = kAccCount * sizeof(unsigned long long);
  nb->spill = static_cast<size_t>(j->sieve_grid) * spill_cap_of(c) * 8;
  nb->queries = s.q.size() * sizeof(Query);
  nb->segpref = s.prefix.size() * sizeof(uint64_t);
  nb->smallq = s.small.size() * sizeof(uint32_t);
  if (s.n_segs == 0) j->plan.passes = 0;  // small-class queries only
  return BX_OK;
}

// What the workspace holds once a job with buffers nb has run: each buffer
// keeps its size or grows to the job's (from zero when `released`).
uint64_t bytes_after(const bx_ctx* c, const JobBufs& nb, bool released) {
  const std::pair<const DevBuf*, size_t> v[] = {{&c->l1, nb.l1},       {&c->l2, nb.l2},
                                                {&c->cnt1, nb.cnt1},   {&c->cnt2, nb.cnt2},
                                                {&c->cand, nb.cand},   {&c->out, nb.out},
                                                {&c->flags, nb.flags}, {&c->acc, nb.acc},
                                                {&c->spill, nb.spill}, {&c->queries, nb.queries},
                                                {&c->segpref, nb.segpref}, {&c->smallq, nb.smallq},
                                                {&c->rad, 0}};
  uint64_t t = 0;
  for (const auto& e : v) t += std::max<uint64_t>(released ? 0 : e.first->bytes, std::max<size_t>(e.second, 256));
  return t;
}

int prepare_job(bx_ctx* c, Segs& s, int batch, uint32_t kinds, hipStream_t st, Job* j) {
  int rc;
  JobBufs nb;
  if ((rc = plan_job(c, s, batch, kinds, j, &nb)) != BX_OK) return rc;
  if ((rc = ensure(c, c->l1, nb.l1)) != BX_OK) return rc;
  if ((rc = ensure(c, c->l2, nb.l2)) != BX_OK) return rc;
  if ((rc = ensure(c, c->cnt1, nb.cnt1)) != BX_OK) return rc;
  if ((rc = ensure(c, c->cnt2, nb.cnt2)) != BX_OK) return rc;
  if ((rc = ensure(c, c->cand, nb.cand)) != BX_OK) return rc;
  if ((rc = ensure(c, c->out, nb.out)) != BX_OK) return rc;
  if ((rc = ensure(c, c->flags, nb.flags)) != BX_OK) return rc;
  if ((rc = ensure(c, c->acc, nb.acc)) != BX_OK) return rc;
  if ((rc = ensure(c, c->spill, nb.spill)) != BX_OK) return rc;
  if ((rc = upload_segs(c, s, st)) != BX_OK) return rc;
  const Plan& plan = j->plan;
  c->stats.b1_bits = plan.b1bits;
  c->stats.b2_bits = plan.b2bits;
  c->stats.l2_entry_bytes = j->compact ? 8u : 12u;
  c->stats.seg_len = c->seg_len;
  c->stats.tile = static_cast<uint32_t>(c->tile);
  return BX_OK;
}

// Counters start at zero; the join kernel clears every group cursor it reads.
int enqueue_init(bx_ctx* c, const Job& j, hipStream_t st) {
  int rc;
  if ((rc = fill_u32(c, c->flags.p, kFlagCount, 0, st)) != BX_OK) return rc;
  if ((rc = fill_u32(c, c->cnt2.p, j.ngsub, 0, st)) != BX_OK) return rc;
  if ((rc = fill_u32(c, c->acc.p, 2 * kAccCount, 0, st)) != BX_OK) return rc;
  return BX_OK;
}

// One pass: keep the keys whose pass hash lies in [ph_lo, ph_hi).  The sieve
// writes them to first-level regions, then each group of G buckets is split
// into partitions and joined.
int enqueue_pass(bx_ctx* c, const Job& j, uint64_t ph_lo, uint64_t ph_hi, hipStream_t st) {
  const Plan& plan = j.plan;
  uint32_t* d_flags = static_cast<uint32_t*>(c->flags.p);
  SieveParams P = base_sieve_params(c, *j.s);
  P.batch = j.batch;
  P.prune = c->prune;
  P.pfilter = !(ph_lo == 0 && ph_hi == (1ull << 32));
  P.ph_lo = ph_lo;
  P.ph_hi = ph_hi;
  P.b1mask = j.B1 - 1;
  P.l1 = static_cast<Entry*>(c->l1.p);
  P.cap1 = plan.cap1;
  P.cnt1 = static_cast<uint32_t*>(c->cnt1.p);
  {
    LaunchTimer t(c, K_SIEVE, st);
    launch_sieve<MODE_KEYS>(c, P, j.sieve_grid, st);
  }
  BX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_counts, dim3(64), dim3(256), 0, st, static_cast<const uint32_t*>(c->cnt1.p), j.n_regions,
                     static_cast<unsigned long long*>(c->acc.p) + kAccEntries);
  BX_HIP(hipGetLastError());
  for (uint32_t first = 0; first < j.B1; first += j.G) {
    PartParams Q;
    Q.l1 = static_cast<const Entry*>(c->l1.p);
    Q.cap1 = plan.cap1;
    Q.cnt1 = static_cast<const uint32_t*>(c->cnt1.p);
    Q.W = j.sieve_grid;
    Q.first = first;
    Q.G = j.G;
    Q.chunks_per_region = j.cpr;
    Q.l2 = static_cast<Entry*>(c->l2.p);
    Q.cap2 = plan.cap2;
    Q.cnt2 = static_cast<uint32_t*>(c->cnt2.p);
    Q.b2shift = plan.b2bits ? kFpBits - plan.b2bits : 0;
    Q.fp_mask = c->fp_mask;
    Q.b2mask = j.B2 - 1;
    Q.gmask = j.gmask;
    Q.flags = d_flags;
    Q.l2c = static_cast<uint64_t*>(c->l2.p);
    Q.idx_bits = j.idx_bits;
    Q.low_mask = j.low_mask;
    {
      LaunchTimer t(c, K_PART, st);
      const dim3 pg(static_cast<uint32_t>(j.part_grid));
      if (c->fp_mask != (1ull << kFpBits) - 1)
        hipLaunchKernelGGL((k_partition<kPartBlock, true, false>), pg, dim3(kPartBlock), 0, st, Q);
      else if (j.compact)
        hipLaunchKernelGGL((k_partition<kPartBlock, false, true>), pg, dim3(kPartBlock), 0, st, Q);
      else
        hipLaunchKernelGGL((k_partition<kPartBlock, false, false>), pg, dim3(kPartBlock), 0, st, Q);
    }
    BX_HIP(hipGetLastError());
    JoinParams J;
    J.l2 = static_cast<const Entry*>(c->l2.p);
    J.cap2 = plan.cap2;
    J.cnt2 = static_cast<uint32_t*>(c->cnt2.p);
    J.n_sub = j.ngsub;
    J.gmask = j.gmask;
    J.cand = static_cast<Cand*>(c->cand.p);
    J.cand_cap = kCandCap;
    J.flags = d_flags;
    J.joined = static_cast<unsigned long long*>(c->acc.p) + kAccJoined;
    J.l2c = static_cast<const uint64_t*>(c->l2.p);
    J.idx_bits = j.idx_bits;
    J.l1 = static_cast<const Entry*>(c->l1.p);
    J.cap1 = plan.cap1;
    J.W = j.sieve_grid;
    J.first = first;
    J.b2mask = j.B2 - 1;
    {
      LaunchTimer t(c, K_JOIN, st);
      if (j.compact)
        hipLaunchKernelGGL((k_join_c<kJoinBlock>), dim3(static_cast<uint32_t>(j.ngsub)), dim3(kJoinBlock), 0, st, J);
      else if (c->join_sort)
        hipLaunchKernelGGL((k_join_sort<kJoinBlock>), dim3(static_cast<uint32_t>(j.ngsub)), dim3(kJoinBlock), 0, st, J);
      else
        hipLaunchKernelGGL((k_join<kJoinBlock>), dim3(static_cast<uint32_t>(j.ngsub)), dim3(kJoinBlock), 0, st, J);
    }
    BX_HIP(hipGetLastError());
  }
  return BX_OK;
}

// The small-query class: one workgroup per query of at most small_max
// integers sieves, tests and joins it in LDS; its candidates join those of the
// passes in the candidate buffer.
int enqueue_small(bx_ctx* c, const Job& j, hipStream_t st) {
  const Segs& s = *j.s;
  if (s.small.empty()) return BX_OK;
  SmallParams P;
  P.queries = static_cast<const Query*>(c->queries.p);
  P.list = static_cast<const uint32_t*>(c->smallq.p);
  P.batch = j.batch;
  P.prune = c->prune;
  P.pp = c->d_pp;
  P.n_pp = static_cast<uint32_t>(c->pp.size());
  const bool big = c->small_max > static_cast<uint32_t>(kTileSmall);
  P.n_dense = c->n_dense[big ? 1 : 0];
  P.dense = c->d_dense[big ? 1 : 0];
  P.fp_mask = c->fp_mask;
  P.cand = static_cast<Cand*>(c->cand.p);
  P.cand_cap = kCandCap;
  P.flags = static_cast<uint32_t*>(c->flags.p);
  P.acc = static_cast<unsigned long long*>(c->acc.p);
  for (uint32_t qi : s.small) {
    const Query& q = s.q[qi];
    if (q.b - q.a < 2 || q.b - q.a > (big ? kTileLarge : kTileSmall))
      return fail(BX_EINTERNAL, "small-class query outside the class bounds");
  }
  const dim3 grid(static_cast<uint32_t>(s.small.size()));
  {
    LaunchTimer t(c, K_SMALL, st);
#define BX_SMALL_LAUNCH(T, B) hipLaunchKernelGGL((k_small<T, B>), grid, dim3(B), 0, st, P)
    if (big) {
      if (c->small_block == 256)
        BX_SMALL_LAUNCH(kTileLarge, 256);
      else if (c->small_block == 512)
        BX_SMALL_LAUNCH(kTileLarge, 512);
      else
        BX_SMALL_LAUNCH(kTileLarge, 1024);
    } else {
      if (c->small_block == 256)
        BX_SMALL_LAUNCH(kTileSmall, 256);
      else if (c->small_block == 512)
        BX_SMALL_LAUNCH(kTileSmall, 512);
      else
        BX_SMALL_LAUNCH(kTileSmall, 1024);
    }
#undef BX_SMALL_LAUNCH
  }
  BX_HIP(hipGetLastError());
  return BX_OK;
}

int enqueue_verify(bx_ctx* c, const Job& j, uint32_t grid, hipStream_t st) {
  VerifyParams V;
  V.cand = static_cast<const Cand*>(c->cand.p);
  V.n_cand = static_cast<const uint32_t*>(c->flags.p) + kFlagCand;
  V.cand_cap = kCandCap;
  V.primes = c->d_primes;
  V.pinv = c->d_pinv;
  V.n_primes = static_cast<uint32_t>(c->primes.size());
  V.queries = static_cast<const Query*>(c->queries.p);
  V.batch = j.batch;
  V.kinds = j.kinds;
  V.third_off = c->third_off;
  V.fp_mask = c->fp_mask;
  V.out = static_cast<OutPair*>(c->out.p);
  V.out_cap = kCandCap;
  V.flags = static_cast<uint32_t*>(c->flags.p);
  {
    LaunchTimer t(c, K_VERIFY, st);
    hipLaunchKernelGGL((k_verify<kVerifyBlock>), dim3(grid), dim3(kVerifyBlock), 0, st, V);
  }
  BX_HIP(hipGetLastError());
  return BX_OK;
}

// The flag words and the 64-bit counters, read with one wait.
int read_flags_acc(bx_ctx* c, uint32_t* fl, unsigned long long* acc, hipStream_t st) {
  BX_HIP(hipMemcpyAsync(fl, c->flags.p, kFlagCount * 4, hipMemcpyDeviceToHost, st));
  BX_HIP(hipMemcpyAsync(acc, c->acc.p, kAccCount * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  BX_HIP(hipStreamSynchronize(st));
  return BX_OK;
}

// Read the verified pairs (flags and counters already read after the last kernel).
int collect_pairs(bx_ctx* c, const uint32_t* fl, const unsigned long long* acc, hipStream_t st,
                  std::vector<OutPair>* result) {
  if (fl[kFlagSpillOverflow]) return fail(BX_EINTERNAL, "sparse-hit spill buffer overflow");
  if (fl[kFlagCand] > kCandCap) return fail(BX_EINTERNAL, "candidate buffer overflow");
  if (fl[kFlagVerifyFail])
    return fail(BX_EINTERNAL, std::to_string(fl[kFlagVerifyFail]) + " candidate pairs failed exact verification");
  c->stats.candidates = fl[kFlagCand];
  c->stats.false_candidates = fl[kFlagFalseCand];
  c->stats.word_matches = fl[kFlagWordMatch];
  const uint32_t n_out = std::min(fl[kFlagOut], kCandCap);
  c->stats.pairs = n_out;
  result->resize(n_out);
  if (n_out) {
    BX_HIP(hipMemcpyAsync(result->data(), c->out.p, n_out * sizeof(OutPair), hipMemcpyDeviceToHost, st));
    BX_HIP(hipStreamSynchronize(st));
  }
  c->stats.entries = acc[kAccEntries];
  c->stats.joined = acc[kAccJoined];
  std::sort(result->begin(), result->end(), [](const OutPair& x, const OutPair& y) {
    if (x.query != y.query) return x.query < y.query;
    if (x.m != y.m) return x.m < y.m;
    return x.n < y.n;
  });
  return BX_OK;
}

// Passes run one at a time with a check after each: a pass whose buckets
// overflow is discarded and run again split in two (one more pass-hash range
// split), so the result never depends on the bucket sizes.
int run_passes_checked(bx_ctx* c, Job& j, hipStream_t st, std::vector<OutPair>* result) {
  int rc;
  if ((rc = enqueue_init(c, j, st)) != BX_OK) return rc;
  if ((rc = enqueue_small(c, j, st)) != BX_OK) return rc;
  std::deque<std::pair<uint64_t, uint64_t>> pending;
  for (uint64_t v = 0; v < j.plan.passes; ++v)
    pending.emplace_back((v << 32) / j.plan.passes, ((v + 1) << 32) / j.plan.passes);
  uint32_t cand_before = 0;
  unsigned long long acc_before[kAccCount] = {0, 0}, acc[kAccCount] = {0, 0};
  uint32_t fl[kFlagCount] = {};
  if (!j.s->small.empty()) {  // a split pass rolls back to what the small class left
    if ((rc = read_flags_acc(c, fl, acc, st)) != BX_OK) return rc;
    cand_before = fl[kFlagCand];
    std::memcpy(acc_before, acc, sizeof(acc));
  }
  while (!pending.empty()) {
    const uint64_t ph_lo = pending.front().first, ph_hi = pending.front().second;
    pending.pop_front();
    if ((rc = enqueue_pass(c, j, ph_lo, ph_hi, st)) != BX_OK) return rc;
    if ((rc = read_flags_acc(c, fl, acc, st)) != BX_OK) return rc;
    c->stats.passes++;
    if (fl[kFlagSpillOverflow]) return fail(BX_EINTERNAL, "sparse-hit spill buffer overflow");
    if (fl[kFlagL1Overflow] || fl[kFlagL2Overflow]) {
      c->stats.retries++;
      if (ph_hi - ph_lo < 2) return fail(BX_EINTERNAL, "bucket overflow on a single pass-hash value");
      uint32_t* d_flags = static_cast<uint32_t*>(c->flags.p);
      uint32_t z[2] = {0, 0};
      BX_HIP(hipMemcpyAsync(d_flags + kFlagL1Overflow, z, sizeof(z), hipMemcpyHostToDevice, st));
      BX_HIP(hipMemcpyAsync(d_flags + kFlagCand, &cand_before, 4, hipMemcpyHostToDevice, st));
      BX_HIP(hipMemcpyAsync(c->acc.p, acc_before, sizeof(acc_before), hipMemcpyHostToDevice, st));
      BX_HIP(hipStreamSynchronize(st));
      const uint64_t mid = ph_lo + (ph_hi - ph_lo) / 2;
      pending.emplace_front(mid, ph_hi);
      pending.emplace_front(ph_lo, mid);
      continue;
    }
    cand_before = fl[kFlagCand];
    std::memcpy(acc_before, acc, sizeof(acc));
  }
  if (cand_before > 0) {  // otherwise the last read is current
    if (cand_before > kCandCap) return fail(BX_EINTERNAL, "candidate buffer overflow");
    if ((rc = enqueue_verify(c, j, std::min<uint32_t>(cand_before, kVerifyGrid), st)) != BX_OK) return rc;
    if ((rc = read_flags_acc(c, fl, acc, st)) != BX_OK) return rc;
  }
  return collect_pairs(c, fl, acc, st, result);
}

// All passes and the verification captured into one HIP graph and launched
// once (instantiated graphs are reused while the launch shapes stay the same).
// Returns 1 in *redo when a bucket overflowed: the caller then falls back to
// the checked path.
int run_passes_graph(bx_ctx* c, Job& j, hipStream_t st, std::vector<OutPair>* result, int* redo) {
  int rc;
  *redo = 0;
  char key[1024];
  // Every launch shape, every option baked into a kernel argument or choice,
  // and every buffer address the graph's kernels use.
  std::snprintf(key, sizeof(key),
                "%u %llu %u %u %u %u %llu %u %d %u %u %d %u %d %d %llx %u %d %zu %d %u %llx %p %p %p %p %p %p %p %p %p %p %p %p %p %p",
                j.plan.passes, static_cast<unsigned long long>(j.plan.cap1), j.plan.cap2, j.plan.b1bits, j.plan.b2bits,
                j.G, static_cast<unsigned long long>(j.s->n_segs), static_cast<uint32_t>(j.s->q.size()), j.batch,
                j.kinds, c->third_off, c->tile, c->seg_len, c->prune, c->join_sort,
                static_cast<unsigned long long>(c->fp_mask), c->small_max, c->small_block, j.s->small.size(),
                static_cast<int>(j.compact), j.idx_bits, static_cast<unsigned long long>(j.low_mask), c->l1.p,
                c->l2.p, c->spill.p, c->cnt1.p, c->cnt2.p, c->cand.p, c->out.p, c->flags.p, c->acc.p, c->queries.p,
                c->segpref.p, c->smallq.p, static_cast<void*>(c->d_pp), static_cast<void*>(c->d_primes));
  if (!c->graph_exec || c->graph_key != key) {
    if (c->graph_exec) {
      BX_HIP(hipGraphExecDestroy(c->graph_exec));
      c->graph_exec = nullptr;
    }
    uint32_t before[6];
    std::memcpy(before, c->stats.launches, sizeof(before));
    BX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    rc = enqueue_init(c, j, st);
    if (rc == BX_OK) rc = enqueue_small(c, j, st);
    for (uint64_t v = 0; rc == BX_OK && v < j.plan.passes; ++v)
      rc = enqueue_pass(c, j, (v << 32) / j.plan.passes, ((v + 1) << 32) / j.plan.passes, st);
    if (rc == BX_OK) rc = enqueue_verify(c, j, kVerifyGrid, st);
    c->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != BX_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    BX_HIP(e);
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BX_HIP(e);
    c->graph_key = key;
    for (int k = 0; k < 6; ++k) c->graph_launches[k] = c->stats.launches[k] - before[k];
  } else {
    for (int k = 0; k < 6; ++k) c->stats.launches[k] += c->graph_launches[k];
  }
  hipEvent_t a = get_event(c), b = get_event(c);
  if (a) BX_HIP(hipEventRecord(a, st));
  BX_HIP(hipGraphLaunch(c->graph_exec, st));
  if (b) BX_HIP(hipEventRecord(b, st));
  uint32_t fl[kFlagCount];
  unsigned long long acc[kAccCount] = {0, 0};
  if ((rc = read_flags_acc(c, fl, acc, st)) != BX_OK) return rc;
  if (a && b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) == hipSuccess) c->stats.graph_ms += ms;
  }
  if (a) c->ev_free.push_back(a);
  if (b) c->ev_free.push_back(b);
  c->stats.passes += j.plan.passes;
  if (fl[kFlagL1Overflow] || fl[kFlagL2Overflow]) {
    *redo = 1;
    return BX_OK;
  }
  return collect_pairs(c, fl, acc, st, result);
}

// The hash-partitioned exact join over all queries of `s`.
int run_search(bx_ctx* c, Segs& s, int batch, uint32_t kinds, std::vector<OutPair>* result, bool use_graph) {
  hipStream_t st = c->stream;
  result->clear();
  int rc = order_after_last(c, st);
  if (rc != BX_OK) return rc;
  rc = mark_done(c, st);  // host-synchronous from here on: the call drains st
  if (rc != BX_OK) return rc;
  make_segs(c, &s, true);
  if (s.n_segs == 0 && s.small.empty()) return BX_OK;
  Job j;
  if ((rc = prepare_job(c, s, batch, kinds, st, &j)) != BX_OK) return rc;
  c->stats.integers = s.n_ints;
  if (use_graph) {
    int redo = 0;
    if ((rc = run_passes_graph(c, j, st, result, &redo)) != BX_OK) return rc;
    if (!redo) return BX_OK;
    c->stats.retries++;
  }
  return run_passes_checked(c, j, st, result);
}

int to_pairs(const std::vector<OutPair>& v, bx_pair** out, size_t* count) {
  *out = nullptr;
  *count = v.size();
  if (v.empty()) return BX_OK;
  bx_pair* p = static_cast<bx_pair*>(std::malloc(v.size() * sizeof(bx_pair)));
  if (!p) return fail(BX_ENOMEM, "host allocation failed");
  for (size_t i = 0; i < v.size(); ++i) p[i] = bx_pair{v[i].m, v[i].n, v[i].kind, v[i].query};
  *out = p;
  return BX_OK;
}

int radicals_into(bx_ctx* c, uint64_t lo, uint64_t hi, uint64_t* dev_out, hipStream_t st, bool clear_flags = true) {
  Segs s;
  s.q.push_back(Query{lo, hi});
  make_segs(c, &s, false);
  if (s.n_segs == 0) return BX_OK;
  int rc;
  if ((rc = upload_segs(c, s, st)) != BX_OK) return rc;
  if ((rc = ensure(c, c->flags, kFlagCount * 4)) != BX_OK) return rc;
  const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(s.n_segs, 2ull * sieve_wg_per_cu(c) * c->n_cu));
  if ((rc = ensure(c, c->spill, static_cast<size_t>(grid) * spill_cap_of(c) * 8)) != BX_OK) return rc;
  if (clear_flags && (rc = fill_u32(c, c->flags.p, kFlagCount, 0, st)) != BX_OK) return rc;
  SieveParams P = base_sieve_params(c, s);
  P.rad_out = dev_out;
  P.rad_lo = lo;
  P.rad_hi = hi;
  {
    LaunchTimer t(c, K_RAD, st);
    launch_sieve<MODE_RAD>(c, P, grid, st);
  }
  BX_HIP(hipGetLastError());
  return BX_OK;
}

// Algorithm 3's schedule over [a, b): chunks C_i of s values overlapping by
// one; C_i's entries go into a table of 4s slots (pairs inside C_i found on
// insertion), then every earlier chunk is sieved again and probes the table.
// The candidates are verified as in the passes.  Work grows with the square
// of the range: it is the paper's design, kept as a baseline.
int run_alg3(bx_ctx* c, uint64_t a, uint64_t b, uint32_t kinds, std::vector<OutPair>* result) {
  hipStream_t st = c->stream;
  result->clear();
  int rc;
  if ((rc = order_after_last(c, st)) != BX_OK) return rc;
  if ((rc = mark_done(c, st)) != BX_OK) return rc;
  const uint64_t s = 1ull << c->a3_log2, step = s - 1;
  const uint64_t n_chunks = (b - a + step - 1) / step;
  const uint64_t slots = 4 * s;
  if ((rc = ensure(c, c->a3tab, slots * sizeof(uint64_t))) != BX_OK) return rc;
  if ((rc = ensure(c, c->rad, (s + 1) * sizeof(uint64_t))) != BX_OK) return rc;
  if ((rc = ensure(c, c->cand, kCandCap * sizeof(Cand))) != BX_OK) return rc;
  if ((rc = ensure(c, c->out, kCandCap * sizeof(OutPair))) != BX_OK) return rc;
  if ((rc = ensure(c, c->flags, kFlagCount * 4)) != BX_OK) return rc;
  if ((rc = ensure(c, c->acc, kAccCount * sizeof(unsigned long long))) != BX_OK) return rc;
  if ((rc = fill_u32(c, c->flags.p, kFlagCount, 0, st)) != BX_OK) return rc;
  if ((rc = fill_u32(c, c->acc.p, 2 * kAccCount, 0, st)) != BX_OK) return rc;
  uint64_t* rad = static_cast<uint64_t*>(c->rad.p);
  A3Params P;
  P.rad = rad;
  P.table = static_cast<uint64_t*>(c->a3tab.p);
  P.tmask = slots - 1;
  P.cand = static_cast<Cand*>(c->cand.p);
  P.cand_cap = kCandCap;
  P.flags = static_cast<uint32_t*>(c->flags.p);
  auto grid_for = [&](uint64_t n) { return static_cast<uint32_t>(std::min<uint64_t>((n + 255) / 256, 8192)); };
  for (uint64_t i = 0; i < n_chunks; ++i) {
    const uint64_t ci = a + i * step, cnt_i = std::min(step, b - ci);  // entries n in [ci, ci + cnt_i)
    hipLaunchKernelGGL(k_fill_u64, dim3(4096), dim3(256), 0, st, P.table, slots, kA3Empty);
    BX_HIP(hipGetLastError());
    if ((rc = radicals_into(c, ci, ci + cnt_i + 1, rad, st, false)) != BX_OK) return rc;
    P.c0 = ci;
    P.count = static_cast<uint32_t>(cnt_i);
    P.n0 = ci;
    {
      LaunchTimer t(c, K_JOIN, st);
      hipLaunchKernelGGL(k_a3_insert, dim3(grid_for(cnt_i)), dim3(256), 0, st, P);
    }
    BX_HIP(hipGetLastError());
    for (uint64_t j = 0; j < i; ++j) {
      const uint64_t cj = a + j * step;  // a full chunk: entries m in [cj, cj + step)
      if ((rc = radicals_into(c, cj, cj + step + 1, rad, st, false)) != BX_OK) return rc;
      P.c0 = cj;
      P.count = static_cast<uint32_t>(step);
      P.n0 = ci;
      {
        LaunchTimer t(c, K_JOIN, st);
        hipLaunchKernelGGL(k_a3_probe, dim3(grid_for(step)), dim3(256), 0, st, P);
      }
      BX_HIP(hipGetLastError());
    }
    c->stats.passes++;
  }
  c->stats.integers = b - a;
  uint32_t fl[kFlagCount];
  unsigned long long acc_f[kAccCount] = {0, 0};
  if ((rc = read_flags_acc(c, fl, acc_f, st)) != BX_OK) return rc;
  if (fl[kFlagSpillOverflow]) return fail(BX_EINTERNAL, "sparse-hit overflow in the radical sieve");
  if (fl[kFlagCand] > kCandCap) return fail(BX_EINTERNAL, "candidate buffer overflow");
  if (fl[kFlagCand] > 0) {
    Job j;
    j.batch = 0;
    j.kinds = kinds;
    if ((rc = enqueue_verify(c, j, std::min<uint32_t>(fl[kFlagCand], kVerifyGrid), st)) != BX_OK) return rc;
    if ((rc = read_flags_acc(c, fl, acc_f, st)) != BX_OK) return rc;
  }
  return collect_pairs(c, fl, acc_f, st, result);
}

// Algorithm 2 over [a, b): radicals in chunks, one list entry (fingerprint of
// S_n, n) per kept n, the list radix-sorted by fingerprint (seven passes of 8
// bits cover the 53), every pair inside each run of equal keys a candidate,
// verified as in the passes.  The list needs 32 bytes per kept integer (keys
// and values, double-buffered): a baseline for ranges that fit in memory.
int run_alg2(bx_ctx* c, uint64_t a, uint64_t b, uint32_t kinds, std::vector<OutPair>* result) {
  hipStream_t st = c->stream;
  result->clear();
  int rc;
  if ((rc = order_after_last(c, st)) != BX_OK) return rc;
  if ((rc = mark_done(c, st)) != BX_OK) return rc;
  Segs s;
  s.q.push_back(Query{a, b});
  make_segs(c, &s, false);
  const uint64_t cap = s.n_keys + 64;  // bound on the kept integers
  const uint64_t chunk = 1ull << 27;
  const uint64_t n_tiles_max = (cap + kRsTile - 1) / kRsTile, m_max = 256 * n_tiles_max;
  const uint64_t nt_max = (m_max + kScanTile - 1) / kScanTile;
  const uint64_t need = 4 * cap * 8 + m_max * 12 + nt_max * 8 + (std::min(chunk, b - a) + 1) * 8;
  if (need + fixed_bytes(c, 0) > c->budget)
    return fail(BX_ENOMEM, "Algorithm 2 needs " + std::to_string(need) + " device bytes for its list, budget " +
                               std::to_string(c->budget));
  for (int k = 0; k < 2; ++k) {
    if ((rc = ensure(c, c->a2k[k], cap * 8)) != BX_OK) return rc;
    if ((rc = ensure(c, c->a2v[k], cap * 8)) != BX_OK) return rc;
  }
  if ((rc = ensure(c, c->a2hist, m_max * 4)) != BX_OK) return rc;
  if ((rc = ensure(c, c->a2offs, m_max * 8)) != BX_OK) return rc;
  if ((rc = ensure(c, c->a2tot, nt_max * 8)) != BX_OK) return rc;
  if ((rc = ensure(c, c->rad, (std::min(chunk, b - a) + 1) * sizeof(uint64_t))) != BX_OK) return rc;
  if ((rc = ensure(c, c->cand, kCandCap * sizeof(Cand))) != BX_OK) return rc;
  if ((rc = ensure(c, c->out, kCandCap * sizeof(OutPair))) != BX_OK) return rc;
  if ((rc = ensure(c, c->flags, kFlagCount * 4)) != BX_OK) return rc;
  if ((rc = ensure(c, c->acc, kAccCount * sizeof(unsigned long long))) != BX_OK) return rc;
  if ((rc = fill_u32(c, c->flags.p, kFlagCount, 0, st)) != BX_OK) return rc;
  if ((rc = fill_u32(c, c->acc.p, 2 * kAccCount, 0, st)) != BX_OK) return rc;
  uint64_t* rad = static_cast<uint64_t*>(c->rad.p);
  A2KeyParams K;
  K.rad = rad;
  K.qb = b;
  K.prune = c->prune;
  K.fp_mask = c->fp_mask;
  K.keys = static_cast<uint64_t*>(c->a2k[0].p);
  K.vals = static_cast<uint64_t*>(c->a2v[0].p);
  K.cap = cap;
  K.n_out = static_cast<unsigned long long*>(c->acc.p) + kAccEntries;
  K.flags = static_cast<uint32_t*>(c->flags.p);
  for (uint64_t c0 = a; c0 < b; c0 += chunk) {
    const uint64_t cnt = std::min(chunk, b - c0);
    if ((rc = radicals_into(c, c0, c0 + cnt + 1, rad, st, false)) != BX_OK) return rc;
    K.c0 = c0;
    K.count = static_cast<uint32_t>(cnt);
    {
      LaunchTimer t(c, K_SIEVE, st);
      const uint64_t tiles = (cnt + 256 * kA2Items - 1) / (256 * kA2Items);
      hipLaunchKernelGGL((k_a2_keys<256>), dim3(static_cast<uint32_t>(std::min<uint64_t>(tiles, 4096))), dim3(256), 0,
                         st, K);
    }
    BX_HIP(hipGetLastError());
  }
  unsigned long long acc[kAccCount] = {0, 0};
  BX_HIP(hipMemcpyAsync(acc, c->acc.p, sizeof(acc), hipMemcpyDeviceToHost, st));
  BX_HIP(hipStreamSynchronize(st));
  const uint64_t n = acc[kAccEntries];
  if (n > cap) return fail(BX_EINTERNAL, "Algorithm 2: more kept integers than the bound");
  c->stats.integers = b - a;
  c->stats.entries = n;
  // Radix sort of (key, value) by key, least significant digit first.
  const uint64_t n_tiles = (n + kRsTile - 1) / kRsTile, m = 256 * n_tiles;
  const uint64_t nt = (m + kScanTile - 1) / kScanTile;
  int cur = 0;
  for (uint32_t shift = 0; shift < kFpBits && n > 1; shift += 8) {
    const uint64_t* ki = static_cast<const uint64_t*>(c->a2k[cur].p);
    const uint64_t* vi = static_cast<const uint64_t*>(c->a2v[cur].p);
    uint32_t* hist = static_cast<uint32_t*>(c->a2hist.p);
    uint64_t* offs = static_cast<uint64_t*>(c->a2offs.p);
    uint64_t* tot = static_cast<uint64_t*>(c->a2tot.p);
    {
      LaunchTimer t(c, K_PART, st);
      hipLaunchKernelGGL(k_rs_hist, dim3(static_cast<uint32_t>(n_tiles)), dim3(kRsBlock), 0, st, ki, n, shift, hist,
                         n_tiles);
      hipLaunchKernelGGL(k_scan_tiles, dim3(static_cast<uint32_t>(nt)), dim3(kScanBlock), 0, st, hist, m, offs, tot);
      hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, st, tot, nt);
      hipLaunchKernelGGL(k_scan_add, dim3(static_cast<uint32_t>(nt)), dim3(kScanBlock), 0, st, offs, m, tot);
      hipLaunchKernelGGL(k_rs_scatter, dim3(static_cast<uint32_t>(n_tiles)), dim3(kRsBlock), 0, st, ki, vi, n, shift,
                         offs, n_tiles, static_cast<uint64_t*>(c->a2k[cur ^ 1].p),
                         static_cast<uint64_t*>(c->a2v[cur ^ 1].p));
    }
    BX_HIP(hipGetLastError());
    cur ^= 1;
    c->stats.passes++;
  }
  {
    LaunchTimer t(c, K_JOIN, st);
    hipLaunchKernelGGL(k_a2_runs, dim3(static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 8192)))),
                       dim3(256), 0, st, static_cast<const uint64_t*>(c->a2k[cur].p),
                       static_cast<const uint64_t*>(c->a2v[cur].p), n, static_cast<Cand*>(c->cand.p), kCandCap,
                       static_cast<uint32_t*>(c->flags.p));
  }
  BX_HIP(hipGetLastError());
  uint32_t fl[kFlagCount];
  unsigned long long acc_f[kAccCount] = {0, 0};
  if ((rc = read_flags_acc(c, fl, acc_f, st)) != BX_OK) return rc;
  if (fl[kFlagSpillOverflow]) return fail(BX_EINTERNAL, "sparse-hit overflow in the radical sieve");
  if (fl[kFlagL1Overflow]) return fail(BX_EINTERNAL, "Algorithm 2: list overflow");
  if (fl[kFlagCand] > kCandCap) return fail(BX_EINTERNAL, "candidate buffer overflow");
  if (fl[kFlagCand] > 0) {
    Job j;
    j.batch = 0;
    j.kinds = kinds;
    if ((rc = enqueue_verify(c, j, std::min<uint32_t>(fl[kFlagCand], kVerifyGrid), st)) != BX_OK) return rc;
    if ((rc = read_flags_acc(c, fl, acc_f, st)) != BX_OK) return rc;
  }
  rc = collect_pairs(c, fl, acc_f, st, result);
  c->stats.joined = n;
  return rc;
}

// Scratch of bx_radical_segment_dev_noalloc: the counter words, the one-query
// table and the sparse-hit spill of up to kNaGrid sieve workgroups, in one
// fixed device array (every device the library runs on holds its own copy
// until the process ends).  Host code reaches it only through the address
// hipGetSymbolAddress returns on each device.
constexpr uint32_t kNaGrid = 512;   // sieve workgroups of one call at most
constexpr uint32_t kNaSpill = 4096; // spilled sparse hits per workgroup (beyond the LDS list)
constexpr size_t kNaQueryOff = 256, kNaPrefOff = 512, kNaSpillOff = 1024;
constexpr size_t kNaBytes = kNaSpillOff + static_cast<size_t>(kNaGrid) * kNaSpill * sizeof(uint64_t);
static_assert(kFlagCount * sizeof(uint32_t) <= kNaQueryOff && sizeof(Query) <= kNaPrefOff - kNaQueryOff,
              "scratch layout");
static __device__ __align__(256) uint8_t scratch[kNaBytes];

struct NaDevice {
  std::mutex mu;             // serialises the calls that use this device's scratch
  uint8_t* ptr = nullptr;    // device address of `scratch` on this device
};
std::mutex g_na_mu;
std::map<int, std::unique_ptr<NaDevice>> g_na;

// Once per device, with that device current: the device address of its copy
// of the scratch array.
int na_setup(int device, NaDevice** out) {
  std::lock_guard<std::mutex> lk(g_na_mu);
  auto& slot = g_na[device];
  if (!slot) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(BX_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    slot.reset(new NaDevice());
    slot->ptr = static_cast<uint8_t*>(p);
  }
  *out = slot.get();
  return BX_OK;
}

std::mutex g_default_mu;
bx_ctx* g_default = nullptr;

int default_ctx(bx_ctx** out) {
  std::lock_guard<std::mutex> lk(g_default_mu);
  if (!g_default) {
    int rc = bx_create(&g_default, 0, BX_VALUE_LIMIT - 1, 0);
    if (rc != BX_OK) {
      g_default = nullptr;
      return rc;
    }
  }
  *out = g_default;
  return BX_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Serving: one scheduler thread per lane forms batches of admitted requests
// and runs each batch on the lane's own context (own stream, own workspace),
// so the work of different batches overlaps on the device.
struct bx_ctx::Server {
  struct Req {
    uint64_t a, b;
    uint32_t kinds;
    double t_submit = 0, t_done = 0;
    bool done = false;
    int rc = BX_OK;
    std::vector<OutPair> pairs;
  };
  bx_ctx* owner = nullptr;
  uint64_t budget = 0;
  int max_inflight = 2;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  // Device bytes of each lane's workspace: reserved for the batch it runs
  // (what the batch's plan grows it to) or held between batches.  Their sum
  // never exceeds the budget.
  std::vector<uint64_t> held;
  std::vector<char> busy;  // lane runs a batch
  uint64_t peak = 0, admitted = 0, batches = 0, mem_waits = 0, releases = 0;
  uint32_t max_batch = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<bx_ctx*> lanes;
};

namespace {

uint64_t workspace_bytes(const bx_ctx* c) {
  uint64_t t = 0;
  for (const DevBuf* b : {&c->l1, &c->l2, &c->cnt1, &c->cnt2, &c->cand, &c->out, &c->flags, &c->spill, &c->queries,
                          &c->segpref, &c->rad, &c->acc, &c->smallq})
    t += b->bytes;
  return t;
}

void release_workspace(bx_ctx* c) {
  std::lock_guard<std::mutex> lk(c->mu);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : {&c->l1, &c->l2, &c->cnt1, &c->cnt2, &c->cand, &c->out, &c->flags, &c->spill, &c->queries,
                    &c->segpref, &c->rad, &c->acc, &c->smallq})
    free_buf(*b);
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
}

// The workspace the lane context c would hold after running the batch of
// queries q (released first or not), or the bare need (`released` = true).
// *passes receives the number of hash passes its plan takes.
int batch_bytes(bx_ctx* c, const std::vector<Query>& q, bool released, uint64_t* bytes, uint32_t* passes = nullptr) {
  Segs s;
  s.q = q;
  make_segs(c, &s, true);
  *bytes = 0;
  if (passes) *passes = 1;
  if (s.n_segs == 0 && s.small.empty()) return BX_OK;
  Job j;
  JobBufs nb;
  const int rc = plan_job(c, s, 1, BX_BOTH, &j, &nb);
  if (rc != BX_OK) return rc;
  *bytes = bytes_after(c, nb, released);
  if (passes) *passes = std::max<uint32_t>(1, j.plan.passes);
  return BX_OK;
}

void serve_worker(bx_ctx::Server* S, int lane) {
  bx_ctx* c = S->lanes[lane];
  for (;;) {
    std::vector<uint64_t> batch;
    bool release_first = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty()) return;
      uint64_t others = 0;
      for (int l = 0; l < S->max_inflight; ++l)
        if (l != lane) others += S->held[l];
      // Admit queued requests in arrival order while the lanes' workspaces,
      // this one grown to what the batch's plan needs, stay within the budget,
      // and while the batch needs no more hash passes than its first request
      // (a batch that re-sieves more often is better split).
      std::vector<Query> q;
      uint64_t reserve = 0;
      uint32_t p_first = 1;
      while (!S->queue.empty() && batch.size() < kMaxQueries) {
        const auto& r = *S->reqs[S->queue.front()];
        q.push_back(Query{r.a, r.b});
        uint64_t grown = 0, bare = 0;
        uint32_t passes = 1;
        if (batch_bytes(c, q, false, &grown, &passes) != BX_OK) grown = UINT64_MAX;
        if (batch.empty()) p_first = passes;
        if (!batch.empty() && passes > p_first) {
          q.pop_back();
          break;
        }
        if (others + grown <= S->budget) {
          reserve = grown;
        } else if (batch.empty() && batch_bytes(c, q, true, &bare) == BX_OK && others + bare <= S->budget) {
          reserve = bare;  // fits once this lane's own workspace is released
          release_first = true;
        } else {
          q.pop_back();
          break;
        }
        batch.push_back(S->queue.front());
        S->queue.pop_front();
        if (release_first) break;
      }
      if (batch.empty()) {
        // No room: the other lanes hold the budget.  An idle lane lets its
        // workspace go, so that busy lanes finishing their batches (which
        // then find the queue waiting) eventually leave room.
        S->mem_waits++;
        if (S->held[lane] > 0) {
          S->held[lane] = 0;
          lk.unlock();
          release_workspace(c);
          lk.lock();
          S->releases++;
          S->cv.notify_all();
        } else {
          S->cv.wait_for(lk, std::chrono::milliseconds(1));
        }
        continue;
      }
      S->held[lane] = reserve;
      S->busy[lane] = 1;
      uint64_t total = 0;
      for (uint64_t h : S->held) total += h;
      S->peak = std::max(S->peak, total);
      S->admitted += batch.size();
      S->batches++;
      S->max_batch = std::max<uint32_t>(S->max_batch, static_cast<uint32_t>(batch.size()));
      if (release_first) S->releases++;
    }
    if (release_first) release_workspace(c);
    Segs s;
    std::vector<uint32_t> kinds;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (uint64_t t : batch) {
        auto& r = *S->reqs[t];
        s.q.push_back(Query{r.a, r.b});
        kinds.push_back(r.kinds);
      }
    }
    std::vector<OutPair> res;
    int rc;
    uint64_t after = 0;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      reset_stats(c);
      uint32_t kall = 0;  // every kind any request of the batch asks for
      for (uint32_t k : kinds) kall |= k;
      rc = run_search(c, s, 1, kall, &res, c->graph_batch != 0);
      (void)hipStreamSynchronize(c->stream);
      collect_timings(c);
      after = workspace_bytes(c);
    }
    const double t_done = now_s();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (size_t i = 0; i < batch.size(); ++i) {
        auto& r = *S->reqs[batch[i]];
        r.rc = rc;
        r.t_done = t_done;
        r.done = true;
      }
      for (const auto& p : res) {
        auto& r = *S->reqs[batch[p.query]];
        const uint32_t base = p.kind & BX_BOTH;
        const bool three = (r.kinds & BX_THIRD) && (p.kind & BX_THIRD);
        if ((r.kinds & base) || three) r.pairs.push_back(OutPair{p.m, p.n, three ? p.kind : base, 0});
      }
      // What the lane holds now (at most what was reserved for the batch).
      S->held[lane] = std::min(after, S->held[lane]);
      S->busy[lane] = 0;
    }
    S->cv.notify_all();
  }
}

}  // namespace

extern "C" {

int bx_create(bx_ctx** out, int device, uint64_t hi_max, uint64_t hbm_budget_bytes) {
  if (!out) return fail(BX_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  if (hi_max < 2 || hi_max >= BX_VALUE_LIMIT) return fail(BX_ERANGE, "hi_max must be in [2, 2^42)");
  int ndev = 0;
  BX_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(BX_EINVAL, "no HIP device " + std::to_string(device));
  BX_HIP(hipSetDevice(device));
  std::unique_ptr<bx_ctx> c(new bx_ctx());
  c->device = device;
  c->hi_max = hi_max;
  hipDeviceProp_t prop;
  BX_HIP(hipGetDeviceProperties(&prop, device));
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->arch = prop.gcnArchName;
  const size_t colon = c->arch.find(':');
  if (colon != std::string::npos) c->arch.resize(colon);
  BX_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
  c->stream = c->own_stream;
  size_t free_b = 0, total_b = 0;
  BX_HIP(hipMemGetInfo(&free_b, &total_b));
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : static_cast<uint64_t>(0.85 * static_cast<double>(free_b));
  int rc = build_tables(c.get());
  if (rc != BX_OK) return rc;
  NaDevice* na = nullptr;
  if ((rc = na_setup(device, &na)) != BX_OK) return rc;
  c->na = na;
  *out = c.release();
  return BX_OK;
}

void bx_destroy(bx_ctx* c) {
  if (!c) return;
  bx_serve_stop(c);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : {&c->l1, &c->l2, &c->cnt1, &c->cnt2, &c->cand, &c->out, &c->flags, &c->spill, &c->queries,
                    &c->segpref, &c->rad, &c->acc, &c->a3tab, &c->smallq, &c->a2k[0], &c->a2k[1], &c->a2v[0],
                    &c->a2v[1], &c->a2hist, &c->a2offs, &c->a2tot})
    free_buf(*b);
  if (c->d_primes) (void)hipFree(c->d_primes);
  if (c->d_pinv) (void)hipFree(c->d_pinv);
  if (c->d_pp) (void)hipFree(c->d_pp);
  for (DenseTab* d : c->d_dense)
    if (d) (void)hipFree(d);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  reset_stats(c);
  for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
  if (c->last_done) (void)hipEventDestroy(c->last_done);
  if (c->pin_ev) (void)hipEventDestroy(c->pin_ev);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

int bx_set_stream(bx_ctx* c, void* s) {
  if (!c) return fail(BX_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  c->stream = s ? static_cast<hipStream_t>(s) : c->own_stream;
  return BX_OK;
}

int bx_set_option(bx_ctx* c, const char* name, int64_t v) {
  if (!c || !name) return fail(BX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  const std::string n(name);
  if (n == "passes") {
    if (v < 0 || v > 4096) return fail(BX_EINVAL, "passes must be in [0, 4096]");
    c->force_passes = static_cast<int>(v);
  } else if (n == "seg_len") {
    if (v == 0) v = kDefaultSegLen;
    if (v < kTileLarge || v % kTileLarge || v > (1 << 24))
      return fail(BX_EINVAL, "seg_len must be a multiple of 8192 in [8192, 2^24]");
    c->seg_len = static_cast<uint32_t>(v);
  } else if (n == "timing") {
    c->timing = v != 0;
  } else if (n == "tile") {
    if (v != 0 && v != kTileSmall && v != kTileLarge) return fail(BX_EINVAL, "tile must be 0, 2048 or 8192");
    c->tile = v == 0 ? kTileDefault : static_cast<int>(v);
  } else if (n == "schedule") {
    if (v < 0 || v > 2)
      return fail(BX_EINVAL, "schedule must be 0 (hash-partitioned passes), 1 (Algorithm 3) or 2 (Algorithm 2)");
    c->schedule = static_cast<int>(v);
  } else if (n == "a3_chunk_log2") {
    if (v == 0) v = 27;
    if (v < 10 || v > 27) return fail(BX_EINVAL, "a3_chunk_log2 must be in [10, 27]");
    c->a3_log2 = static_cast<uint32_t>(v);
  } else if (n == "graph") {
    c->graph_batch = v != 0;
  } else if (n == "prune") {
    c->prune = v != 0;
  } else if (n == "join") {
    if (v != 0 && v != 1) return fail(BX_EINVAL, "join must be 0 (hash) or 1 (sort)");
    c->join_sort = static_cast<int>(v);
  } else if (n == "fp_bits") {
    if (v != 0 && (v < 12 || v > static_cast<int64_t>(kFpBits)))
      return fail(BX_EINVAL, "fp_bits must be 0 or in [12, 53]");
    const uint64_t all = (1ull << kFpBits) - 1;
    c->fp_mask = (v == 0 || v >= 42) ? all : (all & ~((1ull << 42) - 1)) | ((1ull << v) - 1);
  } else if (n == "third_offset") {
    if (v < 0 || v > 64) return fail(BX_EINVAL, "third_offset must be in [0, 64]");
    c->third_off = static_cast<uint32_t>(v);
  } else if (n == "group") {
    if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8) return fail(BX_EINVAL, "group must be 0, 1, 2, 4 or 8");
    c->force_group = static_cast<int>(v);
  } else if (n == "submit_wait") {
    c->submit_wait = v != 0;
  } else if (n == "compact") {
    if (v < 0 || v > 1) return fail(BX_EINVAL, "compact must be 0 or 1");
    c->compact = static_cast<int>(v);
  } else if (n == "compact_fp_bits") {
    if (v != 0 && (v < 12 || v > 40)) return fail(BX_EINVAL, "compact_fp_bits must be 0 or in [12, 40]");
    c->compact_fp_bits = static_cast<uint32_t>(v);
  } else if (n == "small_max") {
    if (v < 0 || v > static_cast<int64_t>(kSmallMaxLen)) return fail(BX_EINVAL, "small_max must be in [0, 8192]");
    c->small_max = static_cast<uint32_t>(v);
  } else if (n == "small_block") {
    if (v != 0 && v != 256 && v != 512 && v != 1024) return fail(BX_EINVAL, "small_block must be 0, 256, 512 or 1024");
    c->small_block = v == 0 ? 1024 : static_cast<int>(v);
  } else if (n == "b1_bits") {
    if (v > 10) return fail(BX_EINVAL, "b1_bits <= 10");
    c->force_b1 = v == 0 ? -1 : static_cast<int>(v);
  } else if (n == "b2_bits") {
    if (v > 11) return fail(BX_EINVAL, "b2_bits <= 11");
    c->force_b2 = v == 0 ? -1 : static_cast<int>(v);
  } else {
    return fail(BX_EINVAL, "unknown option " + n);
  }
  return BX_OK;
}

int bx_get_stats(bx_ctx* c, bx_stats* out) {
  if (!c || !out) return fail(BX_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  *out = c->stats;
  return BX_OK;
}

int bx_radical_segment(bx_ctx* c, uint64_t lo, uint64_t hi, uint64_t* out) {
  if (!c) return fail(BX_EINVAL, "ctx is NULL");
  if (lo == 0 || hi < lo) return fail(BX_EINVAL, "need 1 <= lo <= hi");
  if (hi > lo && !out) return fail(BX_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  const double t0 = now_s();
  reset_stats(c);
  int rc = check_query(c, lo, hi, 0);
  if (rc != BX_OK) return rc;
  if (hi == lo) return BX_OK;
  BX_HIP(hipSetDevice(c->device));
  if ((rc = order_after_last(c, c->stream)) != BX_OK) return rc;
  if ((rc = ensure(c, c->rad, (hi - lo) * 8)) != BX_OK) return rc;
  if ((rc = radicals_into(c, lo, hi, static_cast<uint64_t*>(c->rad.p), c->stream)) != BX_OK) return rc;
  if ((rc = mark_done(c, c->stream)) != BX_OK) return rc;
  BX_HIP(hipMemcpyAsync(out, c->rad.p, (hi - lo) * 8, hipMemcpyDeviceToHost, c->stream));
  BX_HIP(hipStreamSynchronize(c->stream));
  collect_timings(c);
  c->stats.integers = hi - lo;
  c->stats.total_ms = (now_s() - t0) * 1e3;
  return BX_OK;
}

int bx_radical_segment_dev(bx_ctx* c, uint64_t lo, uint64_t hi, uint64_t* dev_out, void* stream) {
  if (!c) return fail(BX_EINVAL, "ctx is NULL");
  if (lo == 0 || hi < lo) return fail(BX_EINVAL, "need 1 <= lo <= hi");
  if (hi > lo && !dev_out) return fail(BX_EINVAL, "dev_out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  reset_stats(c);
  int rc = check_query(c, lo, hi, 0);
  if (rc != BX_OK) return rc;
  if (hi == lo) return BX_OK;
  BX_HIP(hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);  // NULL: the default stream
  if ((rc = order_after_last(c, st)) != BX_OK) return rc;
  // The query tables are uploaded on `st`; the caller synchronises it.
  rc = radicals_into(c, lo, hi, dev_out, st);
  c->stats.integers = hi - lo;
  if (rc == BX_OK) rc = mark_done(c, st);
  return rc;
}

int bx_radical_segment_dev_noalloc(bx_ctx* c, uint64_t lo, uint64_t hi, uint64_t* dev_out, void* stream) {
  if (!c) return fail(BX_EINVAL, "ctx is NULL");
  if (lo == 0 || hi < lo) return fail(BX_EINVAL, "need 1 <= lo <= hi");
  if (hi > lo && !dev_out) return fail(BX_EINVAL, "dev_out is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  reset_stats(c);
  int rc = check_query(c, lo, hi, 0);
  if (rc != BX_OK) return rc;
  if (hi == lo) return BX_OK;
  // The sparse hits of one segment average seg_len * (sum of 1/q over the
  // sparse powers q <= hi); the LDS list and this workgroup's share of the
  // scratch must hold twice that.
  const int which = c->tile == kTileLarge ? 1 : 0;
  const uint32_t first_sparse = c->n_dense[which];
  const size_t top = static_cast<size_t>(
      std::upper_bound(c->pp.begin(), c->pp.end(), hi, [](uint64_t v, const PrimePow& w) { return v < w.q; }) -
      c->pp.begin());
  const double expect = static_cast<double>(c->seg_len) *
                        (c->cum_inv_q[std::max<size_t>(top, first_sparse)] - c->cum_inv_q[first_sparse]);
  const double room = static_cast<double>(hit_cap<kTileLarge>() + kNaSpill);
  if (2.0 * expect > room)
    return fail(BX_ENOMEM, "segment length " + std::to_string(c->seg_len) + " needs about " +
                               std::to_string(static_cast<uint64_t>(expect)) +
                               " sparse hits per segment; the fixed scratch holds " +
                               std::to_string(static_cast<uint64_t>(room)) + " (use bx_radical_segment_dev)");
  BX_HIP(hipSetDevice(c->device));
  NaDevice* na = static_cast<NaDevice*>(c->na);
  std::lock_guard<std::mutex> lk_na(na->mu);
  hipStream_t st = static_cast<hipStream_t>(stream);  // NULL: the default stream
  if ((rc = order_after_last(c, st)) != BX_OK) return rc;
  uint32_t* flags = reinterpret_cast<uint32_t*>(na->ptr);
  Query* q = reinterpret_cast<Query*>(na->ptr + kNaQueryOff);
  uint64_t* pref = reinterpret_cast<uint64_t*>(na->ptr + kNaPrefOff);
  const uint64_t n_segs = (hi - lo + c->seg_len - 1) / c->seg_len;
  const uint32_t grid = static_cast<uint32_t>(
      std::min<uint64_t>({n_segs, kNaGrid, 2ull * sieve_wg_per_cu(c) * static_cast<uint64_t>(c->n_cu)}));
  // The counters start at zero (a fill kernel), the query table is written
  // from kernel arguments.
  if ((rc = fill_u32(c, flags, kFlagCount, 0, st)) != BX_OK) return rc;
  hipLaunchKernelGGL(k_set_query, dim3(1), dim3(64), 0, st, q, pref, lo, hi, n_segs);
  BX_HIP(hipGetLastError());
  SieveParams P;
  std::memset(&P, 0, sizeof(P));
  P.queries = q;
  P.seg_prefix = pref;
  P.n_queries = 1;
  P.n_segs = n_segs;
  P.seg_len = c->seg_len;
  P.pp = c->d_pp;
  P.n_pp = static_cast<uint32_t>(c->pp.size());
  P.n_dense = first_sparse;
  P.dense = c->d_dense[which];
  P.spill = reinterpret_cast<uint64_t*>(na->ptr + kNaSpillOff);
  P.spill_cap = kNaSpill;
  P.flags = flags;
  P.rad_out = dev_out;
  P.rad_lo = lo;
  P.rad_hi = hi;
  c->stats.launches[K_RAD]++;
  launch_sieve<MODE_RAD>(c, P, grid, st);
  BX_HIP(hipGetLastError());
  // The call waits for its kernels: the overflow word is read back, and the
  // next call may reuse the scratch.
  uint32_t overflow = 0;
  BX_HIP(hipMemcpyAsync(&overflow, flags + kFlagSpillOverflow, sizeof(overflow), hipMemcpyDeviceToHost, st));
  BX_HIP(hipStreamSynchronize(st));
  if (c->last_done) {
    BX_HIP(hipEventRecord(c->last_done, st));
    c->last_stream = st;
  }
  c->stats.integers = hi - lo;
  if (overflow)
    return fail(BX_ENOMEM, "sparse-hit scratch overflow: dev_out is incomplete (use bx_radical_segment_dev)");
  return BX_OK;
}

int bx_search_range(bx_ctx* c, uint64_t a, uint64_t b, uint32_t kinds, bx_pair** out, size_t* count) {
  if (!c || !out || !count) return fail(BX_EINVAL, "NULL argument");
  *out = nullptr;
  *count = 0;
  if (kinds < 1 || kinds > 7) return fail(BX_EINVAL, "kinds must be a mask in 1..7");
  std::lock_guard<std::mutex> lk(c->mu);
  const double t0 = now_s();
  reset_stats(c);
  if (a == 0) a = 1;
  if (b <= a + 1) return BX_OK;
  int rc = check_query(c, a, b, kinds);
  if (rc != BX_OK) return rc;
  BX_HIP(hipSetDevice(c->device));
  Segs s;
  s.q.push_back(Query{a, b});
  std::vector<OutPair> res;
  rc = c->schedule == 1   ? run_alg3(c, a, b, kinds, &res)
       : c->schedule == 2 ? run_alg2(c, a, b, kinds, &res)
                          : run_search(c, s, 0, kinds, &res, false);
  (void)hipStreamSynchronize(c->stream);
  collect_timings(c);
  c->stats.total_ms = (now_s() - t0) * 1e3;
  if (rc != BX_OK) return rc;
  return to_pairs(res, out, count);
}

int bx_benelux_search(bx_ctx* c, uint64_t N, uint32_t kinds, bx_pair** out, size_t* count) {
  if (N >= BX_VALUE_LIMIT) return fail(BX_ERANGE, "N too large");
  return bx_search_range(c, 1, N + 1, kinds, out, count);
}

int bx_search_batch(bx_ctx* c, const uint64_t* a, const uint64_t* b, size_t q, uint32_t kinds, bx_pair** out,
                    size_t* offsets) {
  if (!c || !out || !offsets || (q && (!a || !b))) return fail(BX_EINVAL, "NULL argument");
  *out = nullptr;
  if (kinds < 1 || kinds > 7) return fail(BX_EINVAL, "kinds must be a mask in 1..7");
  if (q > kMaxQueries) return fail(BX_EINVAL, "at most 32768 queries per batch");
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->schedule != 0) return fail(BX_EINVAL, "batched calls run the hash-partitioned passes only (schedule 0)");
  const double t0 = now_s();
  reset_stats(c);
  Segs s;
  for (size_t i = 0; i < q; ++i) {
    uint64_t ai = a[i] == 0 ? 1 : a[i], bi = b[i];
    if (bi < ai) bi = ai;
    if (bi - ai > kMaxQueryLen) return fail(BX_EINVAL, "query longer than 2^28");
    if (bi > ai + 1) {
      int rc = check_query(c, ai, bi, kinds);
      if (rc != BX_OK) return rc;
    } else {
      bi = ai;  // fewer than two integers: no pair, no work
    }
    s.q.push_back(Query{ai, bi});
  }
  BX_HIP(hipSetDevice(c->device));
  std::vector<OutPair> res;
  int rc = run_search(c, s, 1, kinds, &res, c->graph_batch != 0);
  (void)hipStreamSynchronize(c->stream);
  collect_timings(c);
  c->stats.total_ms = (now_s() - t0) * 1e3;
  if (rc != BX_OK) return rc;
  size_t k = 0;
  for (size_t i = 0; i < q; ++i) {
    offsets[i] = k;
    while (k < res.size() && res[k].query == i) ++k;
  }
  offsets[q] = res.size();
  size_t cnt = 0;
  return to_pairs(res, out, &cnt);
}

int bx_serve_start(bx_ctx* c, uint64_t budget_bytes, int max_inflight) {
  if (!c) return fail(BX_EINVAL, "ctx is NULL");
  if (c->server) return fail(BX_EINVAL, "server already running");
  if (max_inflight < 1 || max_inflight > 8) return fail(BX_EINVAL, "max_inflight in [1, 8]");
  auto S = std::make_unique<bx_ctx::Server>();
  S->owner = c;
  S->budget = budget_bytes ? budget_bytes : c->budget / 2;
  S->max_inflight = max_inflight;
  S->held.assign(max_inflight, 0);
  S->busy.assign(max_inflight, 0);
  for (int i = 0; i < max_inflight; ++i) {
    bx_ctx* lane = nullptr;
    // A lane may plan with the whole budget; admission keeps the sum in it.
    int rc = bx_create(&lane, c->device, c->hi_max, S->budget);
    if (rc != BX_OK) {
      for (bx_ctx* l : S->lanes) bx_destroy(l);
      return rc;
    }
    // The lanes search as the owner is set up at the start of serving.
    lane->seg_len = c->seg_len;
    lane->tile = c->tile;
    lane->prune = c->prune;
    lane->join_sort = c->join_sort;
    lane->fp_mask = c->fp_mask;
    lane->third_off = c->third_off;
    lane->force_group = c->force_group;
    lane->small_max = c->small_max;
    lane->small_block = c->small_block;
    lane->compact = c->compact;
    lane->compact_fp_bits = c->compact_fp_bits;
    lane->timing = 0;
    lane->graph_batch = 0;  // batch shapes change from batch to batch: no graph reuse
    S->lanes.push_back(lane);
  }
  bx_ctx::Server* raw = S.get();
  c->server = std::move(S);
  for (int i = 0; i < max_inflight; ++i) raw->workers.emplace_back(serve_worker, raw, i);
  return BX_OK;
}

int bx_serve_stop(bx_ctx* c) {
  if (!c || !c->server) return BX_OK;
  {
    std::lock_guard<std::mutex> lk(c->server->mu);
    c->server->stop = true;
  }
  c->server->cv.notify_all();
  for (auto& t : c->server->workers) t.join();
  for (bx_ctx* l : c->server->lanes) bx_destroy(l);
  c->server.reset();
  return BX_OK;
}

int bx_submit(bx_ctx* c, uint64_t a, uint64_t b, uint32_t kinds, uint64_t* ticket) {
  if (!c || !ticket) return fail(BX_EINVAL, "NULL argument");
  if (!c->server) return fail(BX_EINVAL, "server not started");
  if (kinds < 1 || kinds > 7) return fail(BX_EINVAL, "kinds must be a mask in 1..7");
  if (a == 0) a = 1;
  if (b < a) b = a;
  if (b - a > kMaxQueryLen) return fail(BX_EINVAL, "request longer than 2^28");
  if (b > a + 1) {
    int rc = check_query(c, a, b, kinds);
    if (rc != BX_OK) return rc;
  }
  auto* S = c->server.get();
  if (b > a + 1) {
    // The workspace this request needs on a lane by itself (the lanes' plans
    // depend only on options fixed when serving started).
    uint64_t need = 0;
    const int rc = batch_bytes(S->lanes[0], {Query{a, b}}, true, &need);
    if (rc == BX_ENOMEM) return fail(BX_EBUSY, "request cannot be planned within the serving budget: " + g_err);
    if (rc != BX_OK) return rc;
    if (need > S->budget)
      return fail(BX_EBUSY, "request needs " + std::to_string(need) + " device bytes, more than the serving budget " +
                                std::to_string(S->budget));
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (!c->submit_wait) {
      // Admitted now or refused: nothing queued ahead, and an idle lane whose
      // workspace, rebuilt for this request alone (the lane releases its own
      // first when it must), fits beside what the other lanes hold.
      if (!S->queue.empty()) return fail(BX_EBUSY, "requests are queued (submit without waiting)");
      bool room = false;
      for (int l = 0; l < S->max_inflight && !room; ++l) {
        if (S->busy[l]) continue;
        uint64_t others = 0;
        for (int k = 0; k < S->max_inflight; ++k)
          if (k != l) others += S->held[k];
        uint64_t bare = 0;
        if (b <= a + 1 || (batch_bytes(S->lanes[l], {Query{a, b}}, true, &bare) == BX_OK && others + bare <= S->budget))
          room = true;
      }
      if (!room) return fail(BX_EBUSY, "no lane can admit the request now (submit without waiting)");
    }
    const uint64_t t = S->next_ticket++;
    auto r = std::make_unique<bx_ctx::Server::Req>();
    r->a = a;
    r->b = b;
    r->kinds = kinds;
    r->t_submit = now_s();
    S->reqs[t] = std::move(r);
    S->queue.push_back(t);
    *ticket = t;
  }
  S->cv.notify_all();
  return BX_OK;
}

int bx_poll(bx_ctx* c, uint64_t ticket, int* done) {
  if (!c || !done) return fail(BX_EINVAL, "NULL argument");
  if (!c->server) return fail(BX_EINVAL, "server not started");
  auto* S = c->server.get();
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(BX_EINVAL, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return BX_OK;
}

int bx_take_timed(bx_ctx* c, uint64_t ticket, bx_pair** out, size_t* count, double* t_submit, double* t_done) {
  if (!c || !out || !count) return fail(BX_EINVAL, "NULL argument");
  if (!c->server) return fail(BX_EINVAL, "server not started");
  auto* S = c->server.get();
  std::unique_ptr<bx_ctx::Server::Req> r;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(BX_EINVAL, "unknown ticket");
    if (!it->second->done) return fail(BX_EBUSY, "request not finished");
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  if (t_submit) *t_submit = r->t_submit;
  if (t_done) *t_done = r->t_done;
  if (r->rc != BX_OK) return fail(r->rc, "request failed");
  return to_pairs(r->pairs, out, count);
}

int bx_take(bx_ctx* c, uint64_t ticket, bx_pair** out, size_t* count) {
  return bx_take_timed(c, ticket, out, count, nullptr, nullptr);
}

int bx_serve_get_info(bx_ctx* c, bx_serve_info* out) {
  if (!c || !out) return fail(BX_EINVAL, "NULL argument");
  if (!c->server) return fail(BX_EINVAL, "server not started");
  auto* S = c->server.get();
  std::lock_guard<std::mutex> lk(S->mu);
  bx_serve_info v{};
  v.budget_bytes = S->budget;
  v.peak_bytes = S->peak;
  for (uint64_t h : S->held) v.held_bytes += h;
  v.admitted = S->admitted;
  v.batches = S->batches;
  v.max_batch = S->max_batch;
  v.lanes = static_cast<uint32_t>(S->max_inflight);
  v.memory_waits = S->mem_waits;
  v.releases = S->releases;
  *out = v;
  return BX_OK;
}

// One timed setting of the autotuner: the best of `reps` batched runs after
// one warm-up, each checked against the first result seen (*ref).
int tune_one(bx_ctx* c, const uint64_t* a, const uint64_t* b, size_t q, int reps, std::vector<OutPair>* ref,
             bool* have_ref, double* t_best) {
  int rc = BX_OK;
  *t_best = 1e300;
  for (int r = 0; r <= reps && rc == BX_OK; ++r) {
    std::lock_guard<std::mutex> lk(c->mu);
    reset_stats(c);
    Segs s;
    for (size_t i = 0; i < q; ++i) {
      const uint64_t ai = a[i] == 0 ? 1 : a[i];
      uint64_t bi = b[i] < ai ? ai : b[i];
      if (bi - ai > kMaxQueryLen) return fail(BX_EINVAL, "query longer than 2^28");
      if (bi > ai + 1 && (rc = check_query(c, ai, bi, BX_BOTH)) != BX_OK) return rc;
      if (bi <= ai + 1) bi = ai;
      s.q.push_back(Query{ai, bi});
    }
    BX_HIP(hipSetDevice(c->device));
    std::vector<OutPair> res;
    const double t0 = now_s();
    rc = run_search(c, s, 1, BX_BOTH, &res, c->graph_batch != 0);
    (void)hipStreamSynchronize(c->stream);
    const double ms = (now_s() - t0) * 1e3;
    collect_timings(c);
    if (rc != BX_OK) return rc;
    if (!*have_ref) {
      *ref = res;
      *have_ref = true;
    } else if (res.size() != ref->size() ||
               !std::equal(res.begin(), res.end(), ref->begin(), [](const OutPair& x, const OutPair& y) {
                 return x.m == y.m && x.n == y.n && x.kind == y.kind && x.query == y.query;
               })) {
      return fail(BX_EINTERNAL, "autotune: results differ between settings");
    }
    if (r > 0) *t_best = std::min(*t_best, ms);
  }
  return rc;
}

int bx_autotune(bx_ctx* c, const uint64_t* a, const uint64_t* b, size_t q, int reps, const char* path) {
  if (!c || !a || !b || q == 0 || reps < 1) return fail(BX_EINVAL, "bad autotune arguments");
  if (q > kMaxQueries) return fail(BX_EINVAL, "at most 32768 queries per batch");
  const int saved_tile = c->tile, saved_group = c->force_group, saved_sblock = c->small_block;
  const uint32_t saved_seg = c->seg_len, saved_smax = c->small_max;
  struct Best {
    int tile = kTileSmall, group = 8;
    uint32_t seg = kDefaultSegLen;
    uint32_t small_max = kSmallMaxLen;
    int small_block = 1024;
    double ms = 1e300;
  } best;
  std::vector<OutPair> ref;
  bool have_ref = false;
  int rc = BX_OK;
  auto set = [&](int tile, uint32_t seg, int group, uint32_t smax, int sblock) {
    std::lock_guard<std::mutex> lk(c->mu);
    c->tile = tile;
    c->seg_len = seg;
    c->force_group = group;
    c->small_max = smax;
    c->small_block = sblock;
  };
  // The passes' shape first, with the small-query class at its default ...
  for (int tile : {kTileSmall, kTileLarge}) {
    for (uint32_t seg : {1u << 15, 1u << 16, 1u << 17, 1u << 18, 1u << 19}) {
      for (int group : {2, 4, 8}) {
        if (rc != BX_OK) break;
        set(tile, seg, group, saved_smax, saved_sblock);
        double t = 0.0;
        rc = tune_one(c, a, b, q, reps, &ref, &have_ref, &t);
        if (rc == BX_OK && t < best.ms) best = Best{tile, group, seg, saved_smax, saved_sblock, t};
      }
    }
  }
  // ... then the class's cutoff and workgroup size with that shape.
  for (uint32_t smax : {0u, 1024u, 2048u, 4096u, 8192u}) {
    for (int sblock : {256, 512, 1024}) {
      if (rc != BX_OK || (smax == 0 && sblock != 1024)) continue;
      set(best.tile, best.seg, best.group, smax, sblock);
      double t = 0.0;
      rc = tune_one(c, a, b, q, reps, &ref, &have_ref, &t);
      if (rc == BX_OK && t < best.ms) best = Best{best.tile, best.group, best.seg, smax, sblock, t};
    }
  }
  if (rc != BX_OK) {
    set(saved_tile, saved_seg, saved_group, saved_smax, saved_sblock);
    return rc;
  }
  set(best.tile, best.seg, best.group, best.small_max, best.small_block);
  if (path) {
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(BX_EDEVICE, std::string("cannot write ") + path);
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"tile\": %d, \"seg_len\": %u, \"group\": %d, \"small_max\": %u, "
                 "\"small_block\": %d, \"ms\": %.3f}\n",
                 c->arch.c_str(), best.tile, best.seg, best.group, best.small_max, best.small_block, best.ms);
    std::fclose(f);
  }
  return BX_OK;
}

int bx_load_tuning(bx_ctx* c, const char* path) {
  if (!c || !path) return fail(BX_EINVAL, "NULL argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(BX_EINVAL, std::string("cannot read ") + path);
  char buf[1024] = {0};
  const size_t n = std::fread(buf, 1, sizeof(buf) - 1, f);
  std::fclose(f);
  buf[n] = 0;
  const std::string t(buf);
  auto field = [&](const char* name, long long* v) {
    const size_t k = t.find(std::string("\"") + name + "\"");
    if (k == std::string::npos) return false;
    const size_t colon = t.find(':', k);
    if (colon == std::string::npos) return false;
    return std::sscanf(t.c_str() + colon + 1, " %lld", v) == 1;
  };
  const size_t ka = t.find("\"arch\"");
  if (ka != std::string::npos) {
    const size_t q1 = t.find('"', t.find(':', ka));
    const size_t q2 = q1 == std::string::npos ? q1 : t.find('"', q1 + 1);
    if (q1 != std::string::npos && q2 != std::string::npos && t.substr(q1 + 1, q2 - q1 - 1) != c->arch) return BX_OK;
  }
  long long tile = 0, seg = 0, group = 0;
  if (!field("tile", &tile) || !field("seg_len", &seg) || !field("group", &group))
    return fail(BX_EINVAL, std::string("malformed tuning file ") + path);
  int rc;
  if ((rc = bx_set_option(c, "tile", tile)) != BX_OK) return rc;
  if ((rc = bx_set_option(c, "seg_len", seg)) != BX_OK) return rc;
  if ((rc = bx_set_option(c, "group", group)) != BX_OK) return rc;
  // The small-query class fields are optional (files written before the class existed).
  long long smax = 0, sblock = 0;
  if (field("small_max", &smax) && (rc = bx_set_option(c, "small_max", smax)) != BX_OK) return rc;
  if (field("small_block", &sblock) && (rc = bx_set_option(c, "small_block", sblock)) != BX_OK) return rc;
  return BX_OK;
}

double bx_now(void) { return now_s(); }

void bx_free(void* p) { std::free(p); }

const char* bx_last_error(void) { return g_err.c_str(); }

int benelux_search(uint64_t N, uint32_t kinds, bx_pair** out, size_t* count) {
  bx_ctx* c = nullptr;
  int rc = default_ctx(&c);
  if (rc != BX_OK) return rc;
  return bx_benelux_search(c, N, kinds, out, count);
}

int radical_segment(uint64_t lo, uint64_t hi, uint64_t* out) {
  bx_ctx* c = nullptr;
  int rc = default_ctx(&c);
  if (rc != BX_OK) return rc;
  return bx_radical_segment(c, lo, hi, out);
}

}  // extern "C"
