// The tail loop and its fold (k_tail_loop + k_tail_fold, the current kernel text) on the
// CPU SIMT shim: from a seed to the fixpoint, one launch pair after another, each with its
// record bound `jstep` iterations ahead (so that bound stops the loop too), as the host
// loop relaunches it.  Every loop must stop at the fixpoint, at the record bound or with a
// full run T; an iteration that outgrows one block is an error here (the inputs are sized
// to fit).  The result and every iteration's sizes go to the output file.
//   tail_harness <in> <out> <fold grid> <workers> <jstep>
// in:  u64 header (query 0 TC / 1 SG, w, key bytes, |E|, |A0|, |B0|), then the sorted keys
//      of E, of run A0 and of run B0 (u64 each); the seed delta is A0 + B0 (all of Full).
// out: u64 iterations I, then (N, C) of iterations 1..I, |Full|, the sorted keys of Full,
//      then the tail launches and how many stopped at the record bound and at a full T.
#include <hip/hip_runtime.h>
#include "wg_launch.h"
#include <fstream>
#include <iterator>
#include <memory>
namespace wg {
#include "tail.inc"
}
using namespace wg;

template <typename K>
int run(const std::vector<uint64_t>& E64, const std::vector<uint64_t>& A64, const std::vector<uint64_t>& B64,
        int query, int w, uint32_t G, unsigned workers, uint32_t jstep, const char* out_path) {
  const K mask = (K)((K(1) << w) - 1);
  std::vector<K> E(E64.begin(), E64.end());
  const uint64_t rows = 1ull << w;
  std::vector<uint32_t> R(rows + 1), Edst(std::max<size_t>(E.size(), 1));
  for (uint64_t v = 0, i = 0; v <= rows; ++v) {
    while (i < E.size() && (uint64_t)(E[i] >> w) < v) ++i;
    R[v] = (uint32_t)i;
  }
  for (size_t i = 0; i < E.size(); ++i) Edst[i] = (uint32_t)(E[i] & mask);
  const uint64_t cap = 1 << 16;  // candidates, delta and Full capacity (keys)
  std::vector<K> full[2], fullB[2], delta[2], cand[2];
  for (int s = 0; s < 2; ++s) {
    full[s].assign(cap, (K)0x5A5A5A5A);
    fullB[s].assign(cap, (K)0x6B6B6B6B);
    delta[s].assign(cap, (K)0x7C7C7C7C);
    cand[s].assign(cap, (K)0x0D0D0D0D);
  }
  std::copy(A64.begin(), A64.end(), full[0].begin());
  std::copy(B64.begin(), B64.end(), fullB[0].begin());
  std::vector<K> seed(A64.begin(), A64.end());
  seed.insert(seed.end(), B64.begin(), B64.end());
  std::sort(seed.begin(), seed.end());
  std::copy(seed.begin(), seed.end(), delta[0].begin());
  std::vector<K> tail(kTailRunBytes / sizeof(K), (K)0x1E1E1E1E);
  const uint32_t rec_cap = 1 << 14;
  std::vector<IterRec> rec(rec_cap);
  std::memset(rec.data(), 0, sizeof(IterRec) * rec_cap);
  rec[0].N = seed.size();
  rec[0].F = seed.size();
  rec[0].FA = A64.size();
  std::unique_ptr<Ctrl> hold(new Ctrl);
  Ctrl* ctrl = hold.get();
  std::memset(ctrl, 0, sizeof(Ctrl));
  ctrl->cand_cap = cap;
  ctrl->full_cap = cap;
  ctrl->done = seed.empty() ? 1u : 0u;  // (as the seed's compaction leaves it)
  Bufs<K> b;
  std::memset(&b, 0, sizeof(b));
  for (int s = 0; s < 2; ++s) {
    b.cand[s] = cand[s].data();
    b.full[s] = full[s].data();
    b.fullB[s] = fullB[s].data();
    b.delta[s] = delta[s].data();
  }
  b.E = E.data();
  b.R = R.data();
  b.Edst = Edst.data();
  b.rec = rec.data();
  b.tail = tail.data();
  b.dense = (uint32_t)rows;
  uint64_t launches = 0, at_records = 0, at_run = 0;
  while (!ctrl->done) {
    const uint32_t jmax = ctrl->iter + jstep;
    if (jmax + 2 >= rec_cap) {
      printf("FAIL no fixpoint within %u iterations\n", rec_cap - 2);
      return 1;
    }
    if (query == 0)
      simt::launch(1, kSmallSortThreads, [&] { k_tail_loop<K, kJoinTC>(ctrl, b, w, jmax); }, workers);
    else
      simt::launch(1, kSmallSortThreads, [&] { k_tail_loop<K, kJoinSG>(ctrl, b, w, jmax); }, workers);
    simt::launch(G, kBlock, [&] { k_tail_fold<K, kMergeItems>(ctrl, b); }, workers);
    ++launches;
    if (ctrl->overflow || ctrl->limit_hit) {
      printf("FAIL flags overflow=%u limit=%u\n", ctrl->overflow, ctrl->limit_hit);
      return 1;
    }
    if (!ctrl->done) {
      if (ctrl->tail_exit == kTailRecords) ++at_records;
      else if (ctrl->tail_exit == kTailRun) ++at_run;
      else {
        printf("FAIL stopped with exit %u at iteration %u\n", ctrl->tail_exit, ctrl->iter);
        return 1;
      }
    }
  }
  const uint32_t I = ctrl->iter;
  const IterRec fin = rec[I];
  std::vector<uint64_t> res(full[fin.a].begin(), full[fin.a].begin() + fin.FA);
  res.insert(res.end(), fullB[fin.b].begin(), fullB[fin.b].begin() + (fin.F - fin.FA));
  if (!std::is_sorted(res.begin(), res.begin() + fin.FA) || !std::is_sorted(res.begin() + fin.FA, res.end())) {
    printf("FAIL runs A and B are not sorted\n");
    return 1;
  }
  std::sort(res.begin(), res.end());
  std::ofstream o(out_path, std::ios::binary);
  auto put = [&](uint64_t v) { o.write((const char*)&v, 8); };
  put(I);
  for (uint32_t j = 1; j <= I; ++j) {
    put(rec[j].N);
    put(rec[j].C);
  }
  put(res.size());
  o.write((const char*)res.data(), (std::streamsize)(res.size() * 8));
  put(launches);
  put(at_records);
  put(at_run);
  printf("ok iterations=%u full=%zu launches=%llu records=%llu run=%llu\n", I, res.size(),
         (unsigned long long)launches, (unsigned long long)at_records, (unsigned long long)at_run);
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 6) return 2;
  std::ifstream f(argv[1], std::ios::binary);
  uint64_t h[6];
  f.read((char*)h, sizeof(h));
  auto get = [&](uint64_t n) {
    std::vector<uint64_t> v(n);
    f.read((char*)v.data(), (std::streamsize)(n * 8));
    return v;
  };
  const std::vector<uint64_t> E = get(h[3]), A = get(h[4]), B = get(h[5]);
  const uint32_t G = (uint32_t)atoi(argv[3]);
  const unsigned workers = (unsigned)atoi(argv[4]);
  const uint32_t jstep = (uint32_t)atoi(argv[5]);
  return h[2] == 4 ? run<uint32_t>(E, A, B, (int)h[0], (int)h[1], G, workers, jstep, argv[2])
                   : run<uint64_t>(E, A, B, (int)h[0], (int)h[1], G, workers, jstep, argv[2]);
}
