// The segmented sort (k_seg_sort, the current kernel text) on the CPU SIMT shim: keys
// grouped by row in ascending row order, each row's keys in any order; the output must be
// the keys sorted, and no block may split.
//   seg_harness <file> <grid> <workers> <reps>
// file: u64 header (keys, w, key bytes), then the keys.
#include <hip/hip_runtime.h>
#include "wg_launch.h"
#include <fstream>
namespace wg {
#include "seg.inc"
}
using namespace wg;

template <typename K>
int run(const std::vector<K>& in, int w, uint32_t G, unsigned workers) {
  const uint64_t n = in.size();
  std::vector<K> src(in), out(std::max<uint64_t>(n, 1), (K)0x3C3C3C3C);
  std::vector<uint32_t> queue(3 * (n / 1024 + 16));
  Ctrl* ctrl = new Ctrl;
  std::memset(ctrl, 0, sizeof(Ctrl));
  ctrl->cand_n = n;
  simt::launch(G, kSmallSortThreads, [&] {
    k_seg_sort<K>(0, ctrl, &ctrl->cand_n, src.data(), out.data(), w, queue.data(), 0);
  }, workers);
  std::vector<K> want(in);
  std::sort(want.begin(), want.end());
  const bool ok = ctrl->overflow == 0 && std::equal(want.begin(), want.end(), out.begin());
  printf("%s n=%llu ovf=%u\n", ok ? "ok" : "FAIL", (unsigned long long)n, ctrl->overflow);
  delete ctrl;
  return ok ? 0 : 1;
}

int main(int argc, char** argv) {
  std::ifstream f(argv[1], std::ios::binary);
  uint64_t h[3];
  f.read((char*)h, sizeof(h));
  const uint32_t G = (uint32_t)atoi(argv[2]);
  const unsigned workers = (unsigned)atoi(argv[3]);
  const int reps = atoi(argv[4]);
  int bad = 0;
  if (h[2] == 4) {
    std::vector<uint32_t> in(h[0]);
    f.read((char*)in.data(), 4 * h[0]);
    for (int r = 0; r < reps; ++r) bad += run<uint32_t>(in, (int)h[1], G, workers);
  } else {
    std::vector<uint64_t> in(h[0]);
    f.read((char*)in.data(), 8 * h[0]);
    for (int r = 0; r < reps; ++r) bad += run<uint64_t>(in, (int)h[1], G, workers);
  }
  return bad ? 1 : 0;
}
