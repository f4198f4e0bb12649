// Test-only helper: evaluates Philox4x32-10 with two independent library
// implementations (PyTorch's ATen engine and rocRAND's device/host engine),
// both compiled here from their source headers, so the oracle's own Philox can
// be checked against them. Reads lines "c0 c1 c2 c3 k0 k1" from stdin and
// prints "aten0..3 rocrand0..3" per line. rocRAND is only queried when its
// 64-bit element offset does not overflow (c1 < 2^30); otherwise it prints 0s.
#include <ATen/core/PhiloxRNGEngine.h>
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const uint64_t key = k0 | (k1 << 32);
    const uint64_t subseq = c2 | (c3 << 32);
    const uint64_t block = c0 | (c1 << 32);
    at::philox_engine a(key, subseq, block);
    uint32_t av[4];
    for (int i = 0; i < 4; ++i) av[i] = a();
    uint32_t rv[4] = {0, 0, 0, 0};
    if (c1 < (1ull << 30)) {
      rocrand_device::philox4x32_10_engine r(key, subseq, 4 * block);
      for (int i = 0; i < 4; ++i) rv[i] = r();
    }
    std::printf("%u %u %u %u %u %u %u %u\n", av[0], av[1], av[2], av[3], rv[0], rv[1], rv[2], rv[3]);
  }
  return 0;
}
