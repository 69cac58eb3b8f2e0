// Test harness: Philox4x32-10 words from PyTorch's ATen header (an installed,
// independently written source implementation).  Reads records of
// (seed u64, subsequence u64, offset u64) from stdin (binary) and writes the
// four 32-bit words of the first block for each record to stdout (binary).
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>
#include <cstdio>

int main() {
  uint64_t rec[3];
  while (std::fread(rec, sizeof(uint64_t), 3, stdin) == 3) {
    at::philox_engine eng(rec[0], rec[1], rec[2]);
    uint32_t out[4];
    for (int l = 0; l < 4; ++l) out[l] = eng();
    std::fwrite(out, sizeof(uint32_t), 4, stdout);
  }
  return 0;
}
