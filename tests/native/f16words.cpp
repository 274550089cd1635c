// Prints the random words of the binary16 stores (lks::F16Words in
// paper_2112_13930_amd/csrc/lks_sr.hpp) for the seeds first, first + 1, ...,
// first + count - 1: one line per seed, the 19 words word(0..18) in hex.
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "lks_sr.hpp"

int main(int argc, char **argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: f16words FIRST COUNT\n");
    return 2;
  }
  const uint32_t first = (uint32_t)std::strtoul(argv[1], nullptr, 0);
  const long count = std::strtol(argv[2], nullptr, 0);
  for (long i = 0; i < count; ++i) {
    lks::F16Words w(first + (uint32_t)i);
    for (int q = 0; q < 19; ++q) std::printf(q ? " %08x" : "%08x", w.word(q));
    std::printf("\n");
  }
  return 0;
}
