// Batch scheduling of the persistent Sign kernels (the device work queue that
// replaces the paper's host scheduler, Sec. 4.3): task claims, the slot
// assignment of a batch, the retiring of signed tasks and the per-slot offsets
// into the workgroup scratch.  Written without device intrinsics so that the
// same code compiles for the host, where a test replays whole launch schedules
// under AddressSanitizer / UndefinedBehaviorSanitizer with every index checked.
//
// Per workgroup, in LDS: h_task[h] / h_next[h] (task index and its next
// nonce index) for the nh <= hmax held tasks, h_win[h] (smallest passing nonce
// index of the batch, ~0 if none), and for each slot s < G of the batch the
// held task s_h[s] and the nonce index s_att[s] it evaluates.  All five arrays
// hold G entries; hmax <= G <= 64 is the caller's contract.
#pragma once
#include <stddef.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define DIL_HD __host__ __device__ __forceinline__
#else
#define DIL_HD inline
#endif

namespace dil {

constexpr uint32_t SCHED_NONE = 0xFFFFFFFFu;  // h_win of a task with no passing nonce yet

// Append the tasks base, base + 1, ... (at most `want`, none at or past
// `count`) to the held list at index nh.  `base` is the work-queue value that
// the caller's atomic add of `want` returned; the counter may run past count.
// Sets queue_empty once the queue has run dry.  Returns the new nh.
DIL_HD int sched_claim(uint32_t base, uint32_t count, uint32_t want, int nh, uint32_t *h_task, uint32_t *h_next,
                       int &queue_empty) {
  const uint32_t got = base >= count ? 0u : (want < count - base ? want : count - base);
  if (got < want) queue_empty = 1;
  for (uint32_t q = 0; q < got; q++) {
    h_task[nh] = base + q;
    h_next[nh] = 0;
    nh++;
  }
  return nh;
}

// Slots of the next batch: all G while the work queue can still refill the
// workgroup.  Once it has run dry (the tail of the launch) and `tail` > 0, only
// tail slots per held task, rounded up to a multiple of the W wavefronts and
// at most G: the batch's w and check phases, which each wavefront runs slot by
// slot, shorten with it, and the last tasks of a launch do not hold their
// workgroup for full batches of speculative nonces.  0 when nothing is held.
DIL_HD int sched_slots(int nh, int G, int W, int queue_empty, int tail) {
  if (nh <= 0) return 0;
  if (!queue_empty || tail <= 0) return G;
  const int ns = (nh * tail + W - 1) / W * W;
  return ns < G ? ns : G;
}

// Lay out one batch of ns slots (ns <= G; ns >= nh unless ns = 0) over the nh
// held tasks: slot s evaluates held task s mod nh at that task's nonce index
// h_next + s / nh (running counters, no division per slot); every task's
// h_next then moves past the indices handed out and its h_win is cleared.
// Returns ns (0 when nothing is held).
DIL_HD int sched_assign(int nh, int ns, uint32_t *h_next, uint32_t *h_win, uint8_t *s_h, uint32_t *s_att) {
  if (!nh) ns = 0;
  int h = 0;
  uint32_t j = 0;
  for (int s = 0; s < ns; s++) {
    s_h[s] = (uint8_t)h;
    s_att[s] = h_next[h] + j;
    if (++h == nh) {
      h = 0;
      j++;
    }
  }
  for (h = 0; h < nh; h++) {
    h_next[h] += (uint32_t)(ns / nh + (h < ns % nh ? 1 : 0));
    h_win[h] = SCHED_NONE;
  }
  return ns;
}

// The same batch laid out task by task: held task h takes c_h consecutive
// slots (c_h = ns / nh, one more for h < ns mod nh) at its nonce indices
// h_next, h_next + 1, ...; then h_next and h_win as in sched_assign.  A kernel
// that gives each wavefront a contiguous range of slots then keeps most of a
// task's candidates on one wavefront, one after another, so that the task's
// A-hat and secret polynomials are fetched from cache after its first
// candidate.  Returns ns (0 when nothing is held).
DIL_HD int sched_assign_contig(int nh, int ns, uint32_t *h_next, uint32_t *h_win, uint8_t *s_h,
                               uint32_t *s_att) {
  if (!nh) ns = 0;
  int s = 0;
  for (int h = 0; h < nh; h++) {
    const int cnt = ns / nh + (h < ns % nh ? 1 : 0);
    for (int j = 0; j < cnt; j++, s++) {
      s_h[s] = (uint8_t)h;
      s_att[s] = h_next[h] + (uint32_t)j;
    }
    h_next[h] += (uint32_t)cnt;
    h_win[h] = SCHED_NONE;
  }
  return ns;
}

// The range [lo, hi) of a batch's ns slots that wavefront `wave` of W takes
// when each takes a contiguous range: ceil(ns / W) slots each, the last ones
// fewer or none.
DIL_HD void sched_wave_range(int ns, int W, int wave, int &lo, int &hi) {
  const int pw = (ns + W - 1) / W;
  lo = wave * pw;
  hi = lo + pw < ns ? lo + pw : ns;
  if (hi < lo) hi = lo;
}

// Drop the tasks signed in this batch (adding winning index + 1 to
// `sequential`) and those that reached max_attempts without a passing nonce
// (counted in `dropped`), keeping the rest in order.  Returns the new nh.
DIL_HD int sched_retire(int nh, uint32_t *h_task, uint32_t *h_next, const uint32_t *h_win, uint32_t max_attempts,
                        uint64_t &sequential, uint32_t &dropped) {
  int o = 0;
  for (int h = 0; h < nh; h++) {
    if (h_win[h] != SCHED_NONE) {
      sequential += (uint64_t)h_win[h] + 1;
      continue;
    }
    if (h_next[h] >= max_attempts) {
      dropped++;
      continue;
    }
    h_task[o] = h_task[h];
    h_next[o] = h_next[h];
    o++;
  }
  return o;
}

// Element offsets into the persistent kernels' scratch (one region of G slots
// per workgroup; N = 256 coefficients per polynomial).  The workspace carves
// grid * G * L * N words for y, grid * G * K * N for w, grid * G * w1_stride
// bytes for the packed w1 rows and grid * G * sig_stride bytes for staged
// signatures.
struct ScratchIdx {
  size_t G, L, K, w1_stride, sig_stride;
  DIL_HD size_t y(size_t wg, size_t s, size_t i) const { return ((wg * G + s) * L + i) * 256; }
  DIL_HD size_t w(size_t wg, size_t s, size_t i) const { return ((wg * G + s) * K + i) * 256; }
  DIL_HD size_t w1(size_t wg, size_t s) const { return (wg * G + s) * w1_stride; }
  DIL_HD size_t stage(size_t wg, size_t s) const { return (wg * G + s) * sig_stride; }
  // sizes of the four regions for `grid` workgroups (elements / bytes as above)
  DIL_HD size_t y_size(size_t grid) const { return grid * G * L * 256; }
  DIL_HD size_t w_size(size_t grid) const { return grid * G * K * 256; }
  DIL_HD size_t w1_size(size_t grid) const { return grid * G * w1_stride; }
  DIL_HD size_t stage_size(size_t grid) const { return grid * G * sig_stride; }
};

}  // namespace dil
