// Independent Philox4x32 reference for the oracle's pin: PyTorch's own header-only
// engine (ATen/core/PhiloxRNGEngine.h, BSD licence), driven through its public API.
// The engine's seed is the 64-bit key (word 0 low, word 1 high), its subsequence the
// counter words 2-3 and its offset the counter words 0-1; four calls return the block.
// The engine's call operator takes the round count (10 by default).
// Usage: philox_torch_ref N SEED OUTFILE ROUNDS -> N records of 10 uint32 (ctr[4] key[2] out[4]).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

static uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int main(int argc, char **argv) {
  if (argc != 5) return 2;
  const int rounds = std::atoi(argv[4]);
  long n = std::atol(argv[1]);
  uint64_t s = std::strtoull(argv[2], nullptr, 10);
  FILE *f = std::fopen(argv[3], "wb");
  if (!f) return 3;
  for (long i = 0; i < n; i++) {
    uint64_t a = splitmix64(s), b = splitmix64(s), c = splitmix64(s);
    uint32_t rec[10];
    rec[0] = (uint32_t)a; rec[1] = (uint32_t)(a >> 32);
    rec[2] = (uint32_t)b; rec[3] = (uint32_t)(b >> 32);
    if (i % 7 == 0) { rec[2] = (uint32_t)(i % 3); rec[3] = 0; }  // small block numbers
    rec[4] = (uint32_t)c; rec[5] = (uint32_t)(c >> 32);
    if (i % 5 == 0) rec[5] &= 1u;                                // species-like key word
    uint64_t seed = (uint64_t)rec[4] | ((uint64_t)rec[5] << 32);
    uint64_t subseq = (uint64_t)rec[2] | ((uint64_t)rec[3] << 32);
    uint64_t offset = (uint64_t)rec[0] | ((uint64_t)rec[1] << 32);
    at::philox_engine eng(seed, subseq, offset);
    for (int k = 0; k < 4; k++) rec[6 + k] = eng(rounds);
    std::fwrite(rec, sizeof(uint32_t), 10, f);
  }
  std::fclose(f);
  return 0;
}
