// Test helper: evaluates rocRAND's open-source host-callable Philox4x32-10 engine on
// (counter, key) pairs read from stdin and prints the four output words.  Used only to pin
// the oracle's own Philox against an independent implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned a, b, c, d, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subsequence = (unsigned long long)c | ((unsigned long long)d << 32);
    // The engine starts from counter (0, 0, 0, 0); the subsequence fills counter words 2-3
    // and offset / 4 is added to words 0-1, so after the discards below the engine's current
    // block is Philox(ctr = (a, b, c, d), key).  Word 1 is added in four steps of b << 30
    // blocks so that no 64-bit offset overflows.
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * a);
    for (int step = 0; step < 4; ++step) eng.discard(4ull * ((unsigned long long)b << 30));
    unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
