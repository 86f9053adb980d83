// Known-answer generator for Philox4x32-10 taken from rocRAND's engine
// (host-side use of its header).  rocRAND seeds the key with the 64-bit seed
// (low word first) and places the offset/4 in counter words 0-1 and the
// subsequence in counter words 2-3; the first four outputs after
// rocrand_init are the block for that counter.
// Reads lines "seed c0 c1 c2 c3" (c1 < 2^30) from stdin and prints the four
// output words of the block at counter (c0, c1, c2, c3).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_state_philox4x32_10 st;
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    unsigned long long sub = c2 | (c3 << 32);
    rocrand_init(seed, sub, offset, &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
