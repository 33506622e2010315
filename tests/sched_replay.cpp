// Host replay of the persistent Sign kernels' batch scheduling, built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sched.py.
//
// It runs the scheduling code of the loop kernels (paper_2211_12265_amd/csrc/
// batch_sched.h: claims from the shared work queue, slot assignment, retiring) for
// every workgroup of a launch, interleaving the workgroups' batches in a
// seeded random order, and stands in for the candidate evaluation with a
// deterministic pass/fail predicate of (task, nonce index).  The check phase
// follows the multi-wavefront kernel's rule (a slot is skipped once a smaller
// nonce of its task has passed; passes lower h_win with a min), over the slots
// in a random order, as the wavefronts of a workgroup take them concurrently.
//
// Every array the kernels keep in LDS is allocated with exactly G entries so
// the sanitizer sees any overrun, and every index the kernels derive from
// them is checked: held task < nh <= hmax <= G, task < count, slot < G,
// scratch offsets inside the regions carved for `grid` workgroups.  At the
// end each task is signed exactly once at its smallest passing nonce index
// (or dropped at the attempt limit), and the evaluated / sequential counts
// match.
//
// Batches of a workgroup whose queue has run dry take sched_slots' tail
// slots per held task (tail = 0: all G), as the kernels do.  contig = 1 lays
// the batch out task by task (sched_assign_contig) and checks the ranges of
// sched_wave_range: they cover the batch, and each fits one wavefront's 64
// ExpandMask lanes at L streams per slot.
//
// usage: sched_replay G L K count grid hmax p max_attempts seed W tail contig
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <vector>

#include "batch_sched.h"

using namespace dil;

#define CHECK(c)                                                             \
  do {                                                                       \
    if (!(c)) {                                                              \
      fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);        \
      abort();                                                               \
    }                                                                        \
  } while (0)

static uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

struct Wg {
  uint32_t *h_task, *h_next, *h_win, *s_att;
  uint8_t *s_h;
  int nheld = 0, queue_empty = 0;
  bool done = false;
  uint64_t evaluated = 0, sequential = 0;
  uint32_t dropped = 0;
};

int main(int argc, char **argv) {
  if (argc != 13) {
    fprintf(stderr, "usage: %s G L K count grid hmax p max_attempts seed W tail contig\n", argv[0]);
    return 2;
  }
  const int G = atoi(argv[1]), L = atoi(argv[2]), K = atoi(argv[3]);
  const uint32_t count = (uint32_t)strtoul(argv[4], nullptr, 10);
  const size_t grid = (size_t)strtoull(argv[5], nullptr, 10);
  const uint32_t hmax = (uint32_t)strtoul(argv[6], nullptr, 10);
  const double p = atof(argv[7]);
  const uint32_t max_attempts = (uint32_t)strtoul(argv[8], nullptr, 10);
  const uint64_t seed = strtoull(argv[9], nullptr, 10);
  const int W = atoi(argv[10]), tail = atoi(argv[11]), contig = atoi(argv[12]);
  CHECK(G >= 1 && G <= 64 && hmax >= 1 && (int)hmax <= G && grid >= 1);
  CHECK(W >= 1 && G % W == 0 && tail >= 0 && tail <= 64);
  const uint64_t thresh = (uint64_t)(p * 18446744073709551615.0);
  auto passes = [&](uint32_t task, uint32_t nonce) {
    return mix64(seed * 0x9E3779B97F4A7C15ULL ^ ((uint64_t)task << 32 | nonce)) < thresh;
  };
  // scratch offsets as the kernels compute them; the regions as the workspace carves them
  const ScratchIdx si{(size_t)G, (size_t)L, (size_t)K, 1024, 2560};
  const size_t ysz = si.y_size(grid), wsz = si.w_size(grid), w1sz = si.w1_size(grid), stsz = si.stage_size(grid);

  std::vector<Wg> wgs(grid);
  for (auto &w : wgs) {
    w.h_task = new uint32_t[G];
    w.h_next = new uint32_t[G];
    w.h_win = new uint32_t[G];
    w.s_att = new uint32_t[G];
    w.s_h = new uint8_t[G];
  }
  uint32_t queue = 0;  // the work-queue counter (may run past count)
  std::vector<int64_t> winner(count, -1);
  std::vector<uint8_t> dropped_task(count, 0);
  std::mt19937_64 rng(seed);
  std::vector<int> perm(G);
  size_t live = grid;
  uint64_t batches = 0;
  while (live) {
    std::vector<size_t> order;
    for (size_t i = 0; i < grid; i++)
      if (!wgs[i].done) order.push_back(i);
    std::shuffle(order.begin(), order.end(), rng);
    for (size_t wgi : order) {
      Wg &w = wgs[wgi];
      // claim and slot assignment (thread 0 of the workgroup)
      int nh = w.nheld;
      if (!w.queue_empty && nh < (int)hmax) {
        const uint32_t want = hmax - (uint32_t)nh;
        const uint32_t base = queue;
        queue += want;
        nh = sched_claim(base, count, want, nh, w.h_task, w.h_next, w.queue_empty);
      }
      CHECK(nh >= 0 && nh <= (int)hmax);
      w.nheld = nh;
      const int want = sched_slots(nh, G, W, w.queue_empty, tail);
      const int ns = contig ? sched_assign_contig(nh, want, w.h_next, w.h_win, w.s_h, w.s_att)
                            : sched_assign(nh, want, w.h_next, w.h_win, w.s_h, w.s_att);
      CHECK(ns == want && ns <= G);
      if (contig) {
        // task by task: held task indices never decrease along the slots
        for (int s = 1; s < ns; s++) CHECK(w.s_h[s] >= w.s_h[s - 1]);
        int covered = 0;
        for (int wave = 0; wave < W; wave++) {
          int lo = -1, hi = -1;
          sched_wave_range(ns, W, wave, lo, hi);
          CHECK(lo >= 0 && hi >= lo && hi <= ns && (hi - lo) * L <= 64);
          CHECK(hi == lo || lo == covered);
          covered += hi - lo;
        }
        CHECK(covered == ns);
      }
      if (nh && (!w.queue_empty || tail == 0)) CHECK(ns == G);
      if (nh && w.queue_empty && tail > 0) CHECK(ns >= nh && (ns == G || ns % W == 0) && ns >= std::min(G, nh * tail));
      w.evaluated += (uint64_t)ns;
      if (ns == 0) {
        CHECK(nh == 0 && (w.queue_empty || count == 0));
        w.done = true;
        live--;
        continue;
      }
      batches++;
      for (int s = 0; s < ns; s++) {
        CHECK(w.s_h[s] < nh);
        CHECK(w.h_task[w.s_h[s]] < count);
        for (int i = 0; i < L; i++) CHECK(si.y(wgi, s, i) + 256 <= ysz);
        for (int i = 0; i < K; i++) CHECK(si.w(wgi, s, i) + 256 <= wsz);
        CHECK(si.w1(wgi, s) + 1024 <= w1sz && si.stage(wgi, s) + 2560 <= stsz);
      }
      // each held task's slots carry consecutive, increasing nonce indices
      for (int h = 0; h < nh; h++) {
        uint32_t prev = 0;
        bool first = true;
        for (int s = 0; s < ns; s++)
          if (w.s_h[s] == h) {
            CHECK(first || w.s_att[s] == prev + 1);
            prev = w.s_att[s];
            first = false;
          }
        CHECK(!first && prev + 1 == w.h_next[h]);
      }
      // check phase: slots in any order; skip once a smaller nonce passed
      for (int s = 0; s < G; s++) perm[s] = s;
      std::shuffle(perm.begin(), perm.begin() + ns, rng);
      for (int q = 0; q < ns; q++) {
        const int s = perm[q];
        const int h = w.s_h[s];
        if (w.h_win[h] < w.s_att[s]) continue;
        if (passes(w.h_task[h], w.s_att[s])) w.h_win[h] = std::min(w.h_win[h], w.s_att[s]);
      }
      // copy-out: exactly one slot evaluated each winning nonce
      for (int h = 0; h < nh; h++) {
        const uint32_t win = w.h_win[h];
        if (win == SCHED_NONE) continue;
        int hits = 0;
        for (int s = 0; s < ns; s++) hits += (w.s_h[s] == h && w.s_att[s] == win);
        CHECK(hits == 1);
        const uint32_t task = w.h_task[h];
        CHECK(winner[task] < 0);
        winner[task] = win;
      }
      // the tasks this retire drops at the attempt limit
      for (int h = 0; h < nh; h++)
        if (w.h_win[h] == SCHED_NONE && w.h_next[h] >= max_attempts) dropped_task[w.h_task[h]] = 1;
      w.nheld = sched_retire(nh, w.h_task, w.h_next, w.h_win, max_attempts, w.sequential, w.dropped);
      CHECK(w.nheld >= 0 && w.nheld <= nh);
    }
  }
  uint64_t evaluated = 0, sequential = 0, dropped = 0, expect_seq = 0;
  for (auto &w : wgs) {
    evaluated += w.evaluated;
    sequential += w.sequential;
    dropped += w.dropped;
  }
  for (uint32_t t = 0; t < count; t++) {
    if (dropped_task[t]) {
      CHECK(winner[t] < 0);
      for (uint32_t n = 0; n < max_attempts; n++) CHECK(!passes(t, n));
      continue;
    }
    CHECK(winner[t] >= 0);
    uint32_t first = 0;
    while (!passes(t, first)) first++;
    CHECK((uint32_t)winner[t] == first);
    expect_seq += (uint64_t)first + 1;
  }
  CHECK(sequential == expect_seq);
  CHECK(evaluated >= sequential);
  uint64_t ndropped = 0;
  for (uint8_t d : dropped_task) ndropped += d;
  CHECK(ndropped == dropped);
  printf("ok tasks=%u grid=%zu G=%d hmax=%u batches=%llu evaluated=%llu sequential=%llu dropped=%llu\n", count, grid, G,
         hmax, (unsigned long long)batches, (unsigned long long)evaluated, (unsigned long long)sequential,
         (unsigned long long)dropped);
  for (auto &w : wgs) {
    delete[] w.h_task;
    delete[] w.h_next;
    delete[] w.h_win;
    delete[] w.s_att;
    delete[] w.s_h;
  }
  return 0;
}
