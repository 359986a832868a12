// Host checks of the launch plan's index arithmetic (lingam_internal.h), built
// for the CPU by tests/test_plan_host.py.  Prints one line per failed check
// and "ok <checks>" at the end; exits non-zero on any failure.
#include "lingam_internal.h"

#include <cstdint>
#include <cstdio>
#include <vector>

using namespace lg;

namespace {

long g_checks = 0, g_fail = 0;

void expect(bool ok, const char* what, long a = 0, long b = 0, long c = 0, long e = 0) {
  ++g_checks;
  if (!ok && g_fail++ < 20) std::printf("FAIL %s (%ld %ld %ld %ld)\n", what, a, b, c, e);
}

// The all-pairs tile order: [0, nb (nb + 1) / 2) onto the blocks bi <= bj < nb,
// one to one; super-rows of kSuperTile block rows in order; in each, the
// blocks of its diagonal triangle before the blocks to their right.
void check_tiles(int nb) {
  const int64_t T = (int64_t)nb * (nb + 1) / 2;
  std::vector<uint8_t> seen((size_t)nb * nb, 0);
  int last_super = 0;
  bool right_part = false;
  for (int64_t t = 0; t < T; ++t) {
    int bi = -1, bj = -1;
    decode_tile_st((int)t, nb, bi, bj);
    if (!(bi >= 0 && bi <= bj && bj < nb)) {
      expect(false, "tile in the upper triangle", nb, (long)t, bi, bj);
      return;
    }
    uint8_t& s = seen[(size_t)bi * nb + bj];
    expect(s == 0, "tile decoded once", nb, (long)t, bi, bj);
    s = 1;
    const int sup = bi / kSuperTile;
    expect(sup >= last_super, "super-rows in order", nb, (long)t, sup, last_super);
    if (sup != last_super) right_part = false;
    last_super = sup;
    const int r0 = sup * kSuperTile;
    const int h = nb - r0 < kSuperTile ? nb - r0 : kSuperTile;
    const bool in_diag = bj < r0 + h;
    expect(!(right_part && in_diag), "diagonal triangle before the blocks to its right", nb,
           (long)t, bi, bj);
    if (!in_diag) right_part = true;
  }
}

// The sample split of a pair pass: nsplit splits of split_len samples (a
// multiple of the sample quantum) cover [0, n_pad) and the last is not
// empty; no split is shorter than min_iters quanta unless the whole range is;
// never more splits than min_iters allows.
void check_split(int64_t items, int32_t n_pad, int32_t cu, Tune tu) {
  int32_t ns = 0, len = 0;
  split_for(items, n_pad, cu, tu, ns, len);
  const int64_t iters = n_pad / kSampleQuantum;
  expect(ns >= 1 && len >= kSampleQuantum, "a split exists", (long)items, n_pad, ns, len);
  expect(len % kSampleQuantum == 0, "split length in whole quanta", (long)items, n_pad, ns, len);
  expect((int64_t)ns * len >= n_pad, "splits cover the samples", (long)items, n_pad, ns, len);
  expect((int64_t)(ns - 1) * len < n_pad, "last split not empty", (long)items, n_pad, ns, len);
  const int64_t cap = iters >= tu.min_iters ? iters / tu.min_iters : 1;
  expect(ns <= cap, "no more splits than min_iters allows", (long)items, n_pad, ns, (long)cap);
  if (iters >= tu.min_iters)
    expect(len / kSampleQuantum >= tu.min_iters, "splits at least min_iters long", (long)items,
           n_pad, ns, len);
  // workgroups of the largest kind stay in int32: items x splits x 4 quadrant items
  expect((double)items * ns * 4 < 2147483647.0, "workgroup count fits int32", (long)items, n_pad,
         ns, len);
  // the splits stop at about target_per_cu workgroups per CU: items x splits
  // <= items + num_cu x target_per_cu, so a pass of T tiles (2 T items) holds
  // at most T + num_cu x target_per_cu / 2 tile-splits of partial sums (the
  // suspect pass's workspace bound)
  expect(items * ns <= items + (int64_t)cu * tu.target_per_cu, "splits stop near the target",
         (long)items, n_pad, ns, (long)cu * tu.target_per_cu);
  // the most aggressive policy splits the most (the workspace is sized for
  // it): more splits with a larger target, or a smaller min_iters
  if (tu.target_per_cu < kMaxTargetPerCu || tu.min_iters > kMinMinIters) {
    int32_t nsw = 0, lenw = 0;
    split_for(items, n_pad, cu, Tune{kMaxTargetPerCu, kMinMinIters, 4, 4}, nsw, lenw);
    expect(nsw >= ns, "the most aggressive policy splits the most", (long)items, n_pad, ns, nsw);
  }
  // more items over the batch never give a job more splits, so a launch bound
  // computed from one job's items bounds the plan the device makes from the
  // batch's (the suspect pass's bound on the host)
  for (int64_t more : {items + 1, 2 * items, 7 * items + 3}) {
    int32_t ns2 = 0, len2 = 0;
    split_for(more, n_pad, cu, tu, ns2, len2);
    expect(ns2 <= ns, "splits do not grow with the batch's items", (long)items, (long)more, ns,
           ns2);
  }
}

// A step's plan: the FP64 path up to kFp64MaxM active variables, the upper
// triangle of ceil(m / 8) blocks above it, the learned pass's candidates.
void check_step(int32_t d, int32_t t, int32_t K, int32_t min_m) {
  const JobStep s = job_step_base(d, t, K, min_m);
  const int32_t m = d - t;
  if (m < 2) {
    expect(s.m == 0 && kind_count(s, kKSel) == 0, "finished job plans nothing", d, t);
    return;
  }
  expect(s.m == m, "active count", d, t, s.m);
  expect(s.fp64 == (m <= kFp64MaxM), "FP64 path below the threshold", d, t, s.fp64);
  if (!s.fp64) {
    expect((int64_t)s.nblk * kTileVars >= m && (int64_t)(s.nblk - 1) * kTileVars < m,
           "blocks cover the active variables", d, t, s.nblk);
    expect((int64_t)s.ntiles == (int64_t)s.nblk * (s.nblk + 1) / 2, "upper-triangle tiles", d,
           t, s.ntiles);
  }
  const bool learned = K > 0 && m > min_m && !s.fp64;
  expect(s.learned == learned, "learned pass when m > min_m", d, t, s.learned);
  if (learned) {
    const int32_t lo = K < 32 ? K : 32;
    expect(s.k >= lo && s.k <= K, "candidates between min(32, K) and K", d, t, s.k, K);
    expect(s.k <= m, "no more candidates than variables", d, t, s.k, m);
    expect(s.nct == (s.k / kTileVars) * s.nblk, "candidate tiles", d, t, s.nct);
  }
}

// The learned step's second-pass and extension sizes: at most cap_s suspects,
// a multiple of 8, and only while the second pass stays cheaper than the
// full step (2 (K + S) <= m rows); extension columns clamp m - K to ne_max.
void check_bounds(int32_t m, int32_t K, int32_t cap) {
  const int32_t c = suspect_cap(m, K, cap);
  expect(c >= 0 && c % 8 == 0 && c <= cap, "suspect cap a multiple of 8 within the room", m, K,
         cap, c);
  if (c > 0) expect(2 * (K + c) <= m, "second pass cheaper than the full step", m, K, cap, c);
  for (int32_t ne : {0, 8, 128, kMaxExt}) {
    const int32_t e = ext_count(m, K, ne);
    const int32_t want = m - K < 0 ? 0 : (m - K < ne ? m - K : ne);
    expect(e == want, "extension columns", m, K, ne, e);
  }
}

}  // namespace

int main() {
  for (int nb = 1; nb <= 300; ++nb) check_tiles(nb);
  for (int nb : {511, 512, 513, 1023, 1024, 2047, 2048, 4095, 4096}) check_tiles(nb);

  const int64_t item_sizes[] = {1, 2, 7, 45, 90, 1000, 4160, 16512, 1000000, 16781312};
  const int32_t pads[] = {64, 128, 192, 576, 1024, 5056, 8192, 16384, 1 << 20, 1 << 30};
  const int32_t cus[] = {1, 80, 256};
  const int32_t targets[] = {1, 8, 16, kMaxTargetPerCu};
  const int32_t min_iters[] = {kMinMinIters, 8, 16};
  for (int64_t it : item_sizes)
    for (int32_t np : pads)
      for (int32_t cu : cus)
        for (int32_t tg : targets)
          for (int32_t mi : min_iters) check_split(it, np, cu, Tune{tg, mi, 4, 4});

  for (int32_t d : {1, 2, 3, 64, 65, 66, 72, 73, 200, 1024, 4096, 32768})
    for (int32_t K : {0, 16, 64, 256})
      for (int32_t min_m : {0, 128})
        for (int32_t t = 0; t < d; t += (d > 300 ? 97 : 1)) check_step(d, t, K, min_m);

  for (int32_t m = 2; m <= 5000; ++m)
    for (int32_t K : {8, 32, 64, 256})
      for (int32_t cap : {0, 8, 1000, kMaxSuspects}) check_bounds(m, K, cap);

  std::printf("%s %ld checks, %ld failed\n", g_fail ? "FAILED" : "ok", g_checks, g_fail);
  return g_fail ? 1 : 0;
}
