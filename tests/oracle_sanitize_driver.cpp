// Driver for the oracle under the host sanitizers (AddressSanitizer and
// UndefinedBehaviorSanitizer): radicals and searches over small ranges, ranges
// near 2^40 and 2^41, every kinds mask, an empty range.  Built and run by
// tests/test_oracle_sanitizers.py; exits non-zero on the first report.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>
extern "C" {
struct orc_pair { uint64_t m, n; uint32_t kind, reserved; };
uint64_t orc_rad(uint64_t x);
int orc_radicals(uint64_t lo, uint64_t hi, uint64_t* out, int threads);
int orc_search_range_ex(uint64_t a, uint64_t b, uint32_t kinds, uint32_t third_offset, int threads, orc_pair** out,
                        size_t* count, double* t_rad, double* t_join);
void orc_free(void* p);
}
int main() {
  std::vector<uint64_t> r(100000);
  if (orc_radicals(1, 100001, r.data(), 4)) return 1;
  if (orc_radicals((1ull << 40) - 50000, (1ull << 40) + 50000, r.data(), 4)) return 2;
  const uint64_t ranges[][2] = {{1, 2}, {1, 3}, {1, 1 << 16}, {35, 4375}, {(1ull << 41) - 20000, (1ull << 41)}, {5, 5}};
  for (auto& q : ranges)
    for (uint32_t kinds : {1u, 2u, 3u, 7u}) {
      orc_pair* p = nullptr; size_t n = 0; double a = 0, b = 0;
      int rc = orc_search_range_ex(q[0], q[1], kinds, 2, 4, &p, &n, &a, &b);
      if (rc) { std::printf("rc %d\n", rc); return 3; }
      orc_free(p);
    }
  std::printf("ok %llu\n", (unsigned long long)orc_rad(1ull << 40));
  return 0;
}
