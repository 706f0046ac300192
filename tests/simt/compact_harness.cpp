// The fused dedup + set difference (k_compact_local + k_compact_gather, the current kernel
// text, iteration mode) on the CPU SIMT shim, over one input file, `reps` times: the delta
// must equal unique(C) minus (A u B) every time, and no block may split.
//   compact_harness <file> <grid> <workers> <reps> <items 4|8>
// file: u64 header (candidates, |A|, |B|, w, key bytes), then the three key arrays
// (candidates sorted, with duplicates; A and B sorted, distinct, disjoint).
#include <hip/hip_runtime.h>
#include "wg_launch.h"
#include <fstream>
#include <iterator>
namespace wg {
#include "compact.inc"
}
using namespace wg;

template <typename K, int ITEMS>
int run(const std::vector<K>& C, const std::vector<K>& A, const std::vector<K>& B, int w, uint32_t G,
        unsigned workers) {
  const uint64_t n = C.size();
  std::vector<K> cand0(C), cand1(std::max<uint64_t>(n, 1), (K)0x5A5A5A5A), fa(A), fb(B);
  std::vector<K> d0(std::max<uint64_t>(n, 1)), d1(std::max<uint64_t>(n, 1), (K)0x77777777);
  std::vector<uint64_t> bcnt(kScanBlocksMax, 0xDEADBEEFull);
  std::vector<IterRec> rec(4);
  std::memset(rec.data(), 0, sizeof(IterRec) * 4);
  rec[0].F = A.size() + B.size();
  rec[0].FA = A.size();
  Ctrl* ctrl = new Ctrl;
  std::memset(ctrl, 0, sizeof(Ctrl));
  ctrl->cand_n = n;
  ctrl->full_n = rec[0].F;
  ctrl->cand_cap = std::max<uint64_t>(n, 1);
  ctrl->full_cap = rec[0].F + n + 1;
  ctrl->cur = 1;
  Bufs<K> b;
  std::memset(&b, 0, sizeof(b));
  b.cand[0] = cand0.data();
  b.cand[1] = cand1.data();
  b.full[0] = fa.data();
  b.fullB[0] = fb.data();
  b.delta[0] = d0.data();
  b.delta[1] = d1.data();
  b.bcnt = bcnt.data();
  b.rec = rec.data();
  simt::launch(G, kBlock, [&] {
    k_compact_local<K, ITEMS>(ctrl, kModeIter, &ctrl->cand_n, cand0.data(), cand1.data(), b, w, kIterDevice);
  }, workers);
  simt::launch(G, kBlock, [&] {
    k_compact_gather<K, ITEMS>(ctrl, kModeIter, &ctrl->cand_n, cand1.data(), b, kIterDevice, 0u);
  }, workers);
  std::vector<K> u(C);
  u.erase(std::unique(u.begin(), u.end()), u.end());
  std::vector<K> f(A);
  f.insert(f.end(), B.begin(), B.end());
  std::sort(f.begin(), f.end());
  std::vector<K> want;
  std::set_difference(u.begin(), u.end(), f.begin(), f.end(), std::back_inserter(want));
  const uint64_t N = rec[1].N;
  const bool ok = N == want.size() && ctrl->overflow == 0 && std::equal(want.begin(), want.end(), d1.begin());
  printf("%s n=%llu N=%llu want=%zu\n", ok ? "ok" : "FAIL", (unsigned long long)n, (unsigned long long)N,
         want.size());
  delete ctrl;
  return ok ? 0 : 1;
}

template <typename K>
int main_k(std::ifstream& f, const uint64_t* h, uint32_t G, unsigned workers, int reps, int items) {
  std::vector<K> C(h[0]), A(h[1]), B(h[2]);
  f.read((char*)C.data(), sizeof(K) * h[0]);
  f.read((char*)A.data(), sizeof(K) * h[1]);
  f.read((char*)B.data(), sizeof(K) * h[2]);
  int bad = 0;
  for (int r = 0; r < reps; ++r)
    bad += items == 4 ? run<K, 4>(C, A, B, (int)h[3], G, workers) : run<K, 8>(C, A, B, (int)h[3], G, workers);
  return bad ? 1 : 0;
}

int main(int argc, char** argv) {
  std::ifstream f(argv[1], std::ios::binary);
  uint64_t h[5];
  f.read((char*)h, sizeof(h));
  const uint32_t G = (uint32_t)atoi(argv[2]);
  const unsigned workers = (unsigned)atoi(argv[3]);
  const int reps = atoi(argv[4]);
  const int items = atoi(argv[5]);
  return h[4] == 4 ? main_k<uint32_t>(f, h, G, workers, reps, items) : main_k<uint64_t>(f, h, G, workers, reps, items);
}
