// Host-side evaluation of rocRAND's Philox4x32-10 engine, used by the CPU
// test suite as an implementation independent of the oracle's.
// Usage: probe SEED SUBSEQUENCE OFFSET N  -> N 32-bit words, one per line.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  if (argc != 5) return 2;
  unsigned long long seed = strtoull(argv[1], 0, 0);
  unsigned long long subseq = strtoull(argv[2], 0, 0);
  unsigned long long offset = strtoull(argv[3], 0, 0);
  int n = atoi(argv[4]);
  rocrand_state_philox4x32_10 st;
  rocrand_init(seed, subseq, offset, &st);
  for (int i = 0; i < n; ++i) printf("%u\n", rocrand(&st));
  return 0;
}
