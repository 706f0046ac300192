// The row pass and its gather (k_row_diff + k_row_gather, the current kernel text) on the
// CPU SIMT shim, over one input file, `reps` times: the delta must equal the plain set
// difference every time, and no block may split (the shim aborts if it does).
//   row_harness <file> <gather grid> <workers> <reps>
// file: u64 header (candidates, |A|, |B|, w, key bytes), then the three key arrays.
#include <hip/hip_runtime.h>
#include "wg_launch.h"
#include <fstream>
#include <iterator>
namespace wg {
#include "row.inc"
}
using namespace wg;

template <typename K>
int run(const std::vector<K>& C, const std::vector<K>& A, const std::vector<K>& B, int w, uint32_t G,
        unsigned workers) {
  const uint64_t n = C.size();
  std::vector<K> cand0(C), cand1(std::max<uint64_t>(n, 1), (K)0x5A5A5A5A), fa(A), fb(B);
  std::vector<K> d0(std::max<uint64_t>(n, 1)), d1(std::max<uint64_t>(n, 1), (K)0x77777777);
  std::vector<uint64_t> bcnt(std::max<uint32_t>(G, kRowBlocks), 0xDEADBEEFull);
  std::vector<uint64_t> bstart(std::max<uint32_t>(G, kRowBlocks), 0xFEEDFACEull);
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
  b.bstart = bstart.data();
  b.rec = rec.data();
  // the row pass on its own grid (kRowBlocks, every total the gather adds up), the gather on G
  simt::launch(kRowBlocks, kBlock,
               [&] { k_row_diff<K>(0, ctrl, &ctrl->cand_n, cand0.data(), cand1.data(), b, w, kIterDevice); }, workers);
  simt::launch(G, kBlock, [&] { k_row_gather<K>(0, ctrl, cand1.data(), b, kIterDevice); }, workers);
  std::vector<K> u(C);
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  std::vector<K> f(A);
  f.insert(f.end(), B.begin(), B.end());
  std::sort(f.begin(), f.end());
  std::vector<K> want;
  std::set_difference(u.begin(), u.end(), f.begin(), f.end(), std::back_inserter(want));
  const uint64_t N = rec[1].N;
  const bool ok = N == want.size() && ctrl->overflow == 0 && std::equal(want.begin(), want.end(), d1.begin()) &&
                  (ctrl->done != 0) == want.empty();
  printf("%s n=%llu N=%llu want=%zu done=%u\n", ok ? "ok" : "FAIL", (unsigned long long)n, (unsigned long long)N,
         want.size(), ctrl->done);
  delete ctrl;
  return ok ? 0 : 1;
}

int main(int argc, char** argv) {
  std::ifstream f(argv[1], std::ios::binary);
  uint64_t h[5];
  f.read((char*)h, sizeof(h));
  const uint32_t G = (uint32_t)atoi(argv[2]);
  const unsigned workers = (unsigned)atoi(argv[3]);
  const int reps = atoi(argv[4]);
  if (h[4] != 4) return 2;
  std::vector<uint32_t> C(h[0]), A(h[1]), B(h[2]);
  f.read((char*)C.data(), 4 * h[0]);
  f.read((char*)A.data(), 4 * h[1]);
  f.read((char*)B.data(), 4 * h[2]);
  int bad = 0;
  for (int r = 0; r < reps; ++r) bad += run<uint32_t>(C, A, B, (int)h[3], G, workers);
  return bad ? 1 : 0;
}
