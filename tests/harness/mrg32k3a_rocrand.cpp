// Test harness: MRG32k3a outputs from rocRAND's engine header (an installed,
// independently written source implementation with its own jump-ahead
// tables).  Reads records (stream g, substream i, offset) as three u64 from
// stdin (binary); starts from 12345 in all six state words, skips g streams
// (2^127 outputs each), i substreams (2^76 each) and `offset` outputs, and
// writes the next 8 outputs (u32, in [1, m1]) to stdout (binary).
#include <rocrand/rocrand_mrg32k3a.h>

#include <cstdint>
#include <cstdio>

struct Engine : rocrand_device::mrg32k3a_engine {
  void start(uint64_t g, uint64_t i, uint64_t offset) {
    for (int k = 0; k < 3; ++k) {
      m_state.g1[k] = 12345u;
      m_state.g2[k] = 12345u;
    }
    discard_sequence(g);
    discard_subsequence(i);
    discard(offset);
  }
};

int main() {
  uint64_t rec[3];
  Engine e;
  while (std::fread(rec, sizeof(uint64_t), 3, stdin) == 3) {
    e.start(rec[0], rec[1], rec[2]);
    uint32_t out[8];
    for (int l = 0; l < 8; ++l) out[l] = e.next();
    std::fwrite(out, sizeof(uint32_t), 8, stdout);
  }
  return 0;
}
