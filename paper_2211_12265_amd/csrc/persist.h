// Persistent fused Sign kernel with a device-side work queue (Alg. 2 loop).
//
// The paper's host scheduler (Sec. 4.3) refills idle execution units between
// kernel rounds and predicts nonces for unfinished tasks, keeping the valid
// signature with the smallest nonce.  Here the whole rejection loop runs in
// one launch: each workgroup (one wavefront in sg_persist_k, two or four in
// sg_persistw_k) claims tasks from a global atomic counter and owns them
// until they are signed.  Per batch it evaluates G candidate iterations
// ("slots"); when it holds fewer than G tasks, the spare slots evaluate later
// iterations kappa + l*m of the same tasks.  Iterations of one task are
// assigned in increasing order and every earlier iteration has already
// failed, so the smallest passing kappa of the batch is the sequential
// algorithm's answer and becomes the task's signature.  Stages run back to
// back inside the batch:
//   ExpandMask (one lane per stream) -> w = A y per slot (4 groups of 16
//   lanes) -> ctilde and SampleInBall (two lanes per slot) -> checks per slot.
#pragma once
#include "kernels.h"
#include "batch_sched.h"

namespace dil {

template <int LV>
struct PCfg {
  static constexpr int G = 64 / Lv<LV>::L;   // candidate slots per batch: 16 / 12 / 9
  static constexpr int MAX_ATTEMPTS = 16384; // per task; exceeding it flags an error (never reached in practice)
};

// per-workgroup scratch in global memory
struct PScr {
  int32_t *y;    // [P][G][L][256]
  int32_t *w;    // [P][G][K][256]
  uint8_t *w1;   // [P][G][K * W1B rounded to 256]
  uint8_t *stage; // multi-wave kernels only: [P][G][SIG rounded to 256]
};

template <int LV>
__host__ __device__ __forceinline__ size_t w1_stride() {
  return ((size_t)Lv<LV>::K * P<LV>::W1B + 255) & ~(size_t)255;
}
template <int LV>
__host__ __device__ __forceinline__ size_t sig_stride() {
  return ((size_t)P<LV>::SIG + 255) & ~(size_t)255;
}

// Optional per-phase cycle accounting (compile with -DDIL_PHASE_TIMERS): lane 0
// of every workgroup accumulates the s_memtime cycles of each batch phase p and
// adds them at exit to the 64-bit counter at stats words 16 + 2p.
#ifdef DIL_PHASE_TIMERS
#define PHASE_MARK(p)                               \
  do {                                              \
    uint64_t now_ = __builtin_amdgcn_s_memtime();   \
    ph_acc[p] += now_ - ph_t;                       \
    ph_t = now_;                                    \
  } while (0)
#define PHASE_FLUSH()                                                                          \
  do {                                                                                         \
    if (lane == 0)                                                                             \
      for (int p_ = 0; p_ < 5; p_++) atomicAdd((unsigned long long *)&stats[16 + 2 * p_], ph_acc[p_]); \
  } while (0)
#else
#define PHASE_MARK(p) \
  do {                \
  } while (0)
#define PHASE_FLUSH() \
  do {                \
  } while (0)
#endif

// Global-memory stores of a wavefront made visible to its own later loads
// (other lanes of the same wavefront), as between a wavefront's phases when
// no workgroup barrier separates them.
__device__ __forceinline__ void wave_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Claim up to `want` tasks from the work queue with one atomic; they are
// appended to h_task / h_next from index nh.  Sets queue_empty once the queue
// has run dry.  Returns the new number of held tasks.  (The counter may pass
// `count`; it is cleared before every launch.)
__device__ __forceinline__ int claim_tasks(uint32_t *queue, uint32_t count, uint32_t want, int nh, uint32_t *h_task,
                                           uint32_t *h_next, int &queue_empty) {
  return sched_claim(atomicAdd(queue, want), count, want, nh, h_task, h_next, queue_empty);
}

// the scratch offsets of a workgroup shape with G slots per batch
template <int LV>
__device__ __forceinline__ ScratchIdx scratch_idx(int G) {
  return ScratchIdx{(size_t)G, (size_t)Lv<LV>::L, (size_t)Lv<LV>::K, w1_stride<LV>(), sig_stride<LV>()};
}

// Per-workgroup statistics, flushed to the launch's stats words at exit.  It
// lives in LDS, updated by one thread, so that it holds no registers through
// the batch loop (the loop kernels sit at the 256-VGPR limit of two waves per
// SIMD).
struct Tally {
  uint64_t evaluated, sequential;
  uint32_t dropped;
  __device__ void clear() {
    evaluated = sequential = 0;
    dropped = 0;
  }
  __device__ void flush(uint32_t *stats) const {
    if (evaluated) atomicAdd((unsigned long long *)&stats[2], (unsigned long long)evaluated);
    if (sequential) atomicAdd((unsigned long long *)&stats[6], (unsigned long long)sequential);
    if (dropped) atomicAdd(&stats[5], dropped);
  }
};

template <int LV>
struct PersistLds {
  union {
    struct {
      int32_t hat[Lv<LV>::L * HAT_POLY];
      int32_t tr[4 * NTT_LDS_GROUP];
      uint32_t w1buf[Lv<LV>::K * P<LV>::W1B / 4 + 1];
    } wp;
    CheckLds<LV> ck;
  } u;
  int8_t c[PCfg<LV>::G][C_ROW];
  uint32_t ct[PCfg<LV>::G][P<LV>::CT / 4];
  uint32_t bb[PCfg<LV>::G][RATE256 / 4];
  uint32_t h_task[PCfg<LV>::G], h_next[PCfg<LV>::G], h_win[PCfg<LV>::G];
  uint32_t s_att[PCfg<LV>::G];
  uint8_t s_h[PCfg<LV>::G];
  int nheld, nslots, queue_empty;
  Tally tally;
  static_assert(PCfg<LV>::G <= 64, "slot indices are held in bytes and searched with one ballot");
  static_assert(C_ROW >= N && RATE256 / 4 == 34, "challenge rows hold N coefficients, block rows one SHAKE256 block");
  static_assert(sizeof(CheckLds<LV>::sigbuf) >= (size_t)(P<LV>::SIG + 3) / 4 * 4,
                "the staged signature is copied out in whole words");
};

// ws.counters[0] is the work queue (next task to claim).  stats (32-bit words,
// zeroed by the host): [2..3] candidates evaluated (u64), [5] tasks dropped at
// MAX_ATTEMPTS, [6..7] sequential iterations = sum over tasks of (winning
// index + 1) (u64).  hmax: tasks a workgroup holds at a time (1..G).
template <int LV>
__global__ void __launch_bounds__(64) sg_persist_k(Ws ws, PScr sc, uint8_t *sig, uint32_t count, uint32_t hmax,
                                                   uint32_t *stats) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, G = PCfg<LV>::G;
  __shared__ PersistLds<LV> lds;
  const int lane = threadIdx.x, t = lane & 15;
  const size_t wg = blockIdx.x;
  const ScratchIdx si = scratch_idx<LV>(G);
  int32_t *yb = sc.y + si.y(wg, 0, 0);
  int32_t *wb = sc.w + si.w(wg, 0, 0);
  uint8_t *w1b = sc.w1 + si.w1(wg, 0);
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  if (lane == 0) {
    lds.tally.clear();
    lds.nheld = 0;
    lds.queue_empty = 0;
  }
  wave_sync();
#ifdef DIL_PHASE_TIMERS
  uint64_t ph_t = __builtin_amdgcn_s_memtime();
  uint64_t ph_acc[5] = {0, 0, 0, 0, 0};
#endif
  for (;;) {
    // ---- claim tasks and assign the batch's slots ----
    if (lane == 0) {
      int nh = lds.nheld;
      if (!lds.queue_empty && nh < (int)hmax) nh = claim_tasks(ws.counters, count, hmax - nh, nh, lds.h_task,
                                                               lds.h_next, lds.queue_empty);
      lds.nheld = nh;
      const int ns = sched_assign(nh, G, lds.h_next, lds.h_win, lds.s_h, lds.s_att);
      lds.nslots = ns;
      lds.tally.evaluated += (uint64_t)ns;
    }
    wave_sync();
    const int ns = lds.nslots;
    if (ns == 0) break;
    PHASE_MARK(0);
    // ---- ExpandMask: one lane per (slot, i) ----
    if (lane < ns * L) {
      int s = lane / L, i = lane % L;
      uint32_t task = lds.h_task[lds.s_h[s]];
      dev_expand_mask<LV>(ws.rhop + (size_t)task * 64, lds.s_att[s] * (uint32_t)L, i, yb + si.y(0, s, i));
    }
    wave_sync_global();
    PHASE_MARK(1);
    // ---- w = INTT(A NTT(y)) per slot ----
    for (int s = 0; s < ns; s++) {
      uint32_t task = lds.h_task[lds.s_h[s]];
      dev_compute_w<LV>(yb + si.y(0, s, 0), ws.A + kix(ws, task) * K * L * N, wb + si.w(0, s, 0),
                        w1b + si.w1(0, s), lds.u.wp.hat, lds.u.wp.tr + (lane >> 4) * NTT_LDS_GROUP,
                        lds.u.wp.w1buf, ftw, itw, lane);
      wave_sync();
    }
    wave_sync_global();
    PHASE_MARK(2);
    // ---- ctilde and SampleInBall: two lanes per slot ----
    if ((lane >> 1) < ns) {
      const int s = lane >> 1;
      uint32_t task = lds.h_task[lds.s_h[s]];
      dev_challenge_pair<LV>(ws.muw1 + (size_t)task * muw1_stride<LV>(), w1b + si.w1(0, s), lane & 1,
                             lds.ct[s], lds.c[s], lds.bb[s]);
    }
    wave_sync();
    PHASE_MARK(3);
    // ---- checks, in slot order; the first pass of a task is its signature ----
    for (int s = 0; s < ns; s++) {
      int h = lds.s_h[s];
      if (lds.h_win[h] != SCHED_NONE) continue;
      uint32_t task = lds.h_task[h];
      bool ok = dev_check<LV>(lds.c[s], lds.ct[s], yb + si.y(0, s, 0), wb + si.w(0, s, 0),
                              ws.s1h + kix(ws, task) * L * N, ws.s2h + kix(ws, task) * K * N,
                              ws.t0h + kix(ws, task) * K * N, lds.u.ck, ftw, itw, lane);
      if (ok) {
        l2g_bytes(lds.u.ck.sigbuf, P<LV>::SIG, sig + (size_t)task * P<LV>::SIG, lane, 64);
        if (lane == 0) lds.h_win[h] = lds.s_att[s];
      }
      wave_sync();
    }
    PHASE_MARK(4);
    // ---- retire signed tasks ----
    if (lane == 0)
      lds.nheld = sched_retire(lds.nheld, lds.h_task, lds.h_next, lds.h_win, (uint32_t)PCfg<LV>::MAX_ATTEMPTS,
                               lds.tally.sequential, lds.tally.dropped);
    wave_sync();
  }
  if (lane == 0) lds.tally.flush(stats);
  PHASE_FLUSH();
}

}  // namespace dil

namespace dil {

// ---------------------------------------------------------------------------
// Multi-wavefront variant (W = 2 or 4 wavefronts per workgroup).  A workgroup
// holds W * (64 / l) slots per batch.  ExpandMask uses one thread per stream
// over all W waves; w and the checks run per slot, wave w taking slots w,
// w + W, ...; the challenge hashes run on two lanes per slot (keccak_pair.h),
// slots 0..31 on one wave and the rest (at most 32) on the next, while the
// other waves wait at the barrier.  Which waves hash rotates with the
// workgroup and batch index so the SIMDs stay balanced.  Passing candidates
// are staged per slot and the smallest passing nonce of each task is copied
// to the output after a barrier.
//
// At l = 4 (four wavefronts, padded transposes) the batch is laid out task by
// task instead (sched_assign_contig) and wavefront w takes the contiguous
// range sched_wave_range(ns, 4, w): it runs ExpandMask for its own slots
// (one lane per stream, at most 16 slots x 4 streams) and goes on to their w
// phase after a fence of its own, with no workgroup barrier between the two,
// and its w and check phases request their operands early (EARLY in
// dev_compute_w / dev_check).  A task's candidates then follow one another on
// one wavefront and reuse its A-hat and secrets from cache.  The registers
// this takes fit two wavefronts per SIMD at l = 4 only.
// ---------------------------------------------------------------------------
template <int LV, int NW>
struct PCfgW {
  static constexpr int W = NW;
  static constexpr int GW = 64 / Lv<LV>::L;  // slots per wave
  static constexpr int G = W * GW;           // 4 waves: 64 / 48 / 36
  // default tail slots per held task (sched_slots) of the four-wavefront
  // kernel, from interleaved runs at 10,000 tasks: 20 at l = 4 and 12 at l = 5
  // (4% shorter loop kernel than full batches); 0 at l = 7, where the tail
  // kernel's registers no longer fit two wavefronts per SIMD
  static constexpr int TAIL_AUTO = Lv<LV>::L == 4 ? 20 : Lv<LV>::L == 5 ? 12 : 0;
};

template <int LV, int NW>
struct PersistWLds {
  union {
    struct {
      int32_t hat[Lv<LV>::L * HAT_POLY];
      int32_t tr[4 * NTT_LDS_GROUP];
      uint32_t w1buf[Lv<LV>::K * P<LV>::W1B / 4 + 1];
    } wp;
    CheckLds<LV> ck;
  } u[NW];
  int8_t c[PCfgW<LV, NW>::G][C_ROW];
  uint32_t ct[PCfgW<LV, NW>::G][P<LV>::CT / 4];
  uint32_t bb[PCfgW<LV, NW>::G][RATE256 / 4];
  uint32_t h_task[PCfgW<LV, NW>::G], h_next[PCfgW<LV, NW>::G], h_win[PCfgW<LV, NW>::G];
  uint32_t s_att[PCfgW<LV, NW>::G];
  uint8_t s_h[PCfgW<LV, NW>::G];
  int nheld, nslots, queue_empty;
  Tally tally;
  static_assert(PCfgW<LV, NW>::G <= 64, "the winner search takes one slot per lane of one ballot");
  static_assert(C_ROW >= N && RATE256 / 4 == 34, "challenge rows hold N coefficients, block rows one SHAKE256 block");
  static_assert(sizeof(CheckLds<LV>::sigbuf) >= (size_t)(P<LV>::SIG + 3) / 4 * 4,
                "the staged signature is copied in whole words");
};
// two workgroups of the four-wavefront shape per CU (160 KiB of LDS)
static_assert(2 * sizeof(PersistWLds<2, 4>) <= 160 * 1024 && 2 * sizeof(PersistWLds<3, 4>) <= 160 * 1024 &&
                  2 * sizeof(PersistWLds<5, 4>) <= 160 * 1024 && 2 * sizeof(PersistWLds<44, 4>) <= 160 * 1024 &&
                  2 * sizeof(PersistWLds<65, 4>) <= 160 * 1024 && 2 * sizeof(PersistWLds<87, 4>) <= 160 * 1024,
              "four-wavefront loop workgroups must fit two per CU");

// Copy an NB-byte signature from a 4-byte aligned global row to a destination
// row at any byte alignment with one wavefront: each lane requests all the
// source words it needs before storing anything, then funnel-shifts them into
// the destination's word grid (head and tail bytes stored singly).
template <int NB>
__device__ __forceinline__ void copy_sig_row(const uint32_t *src, uint8_t *dst, int lane) {
  constexpr int NWS = (NB + 3) / 4;    // source words
  constexpr int PER = (NWS + 63) / 64;  // destination words per lane (upper bound)
  const int head = (int)((4 - ((uintptr_t)dst & 3)) & 3);
  const int body = (NB - head) >> 2;
  uint32_t lo[PER], hi[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = lane + 64 * q;
    lo[q] = i < NWS ? src[i] : 0u;
    hi[q] = i + 1 < NWS ? src[i + 1] : 0u;
  }
  const uint32_t first = src[0];
  if (lane < head) dst[lane] = (uint8_t)(first >> (8 * lane));
  uint32_t *dw = (uint32_t *)(dst + head);
#pragma unroll
  for (int q = 0; q < PER; q++) {
    const int i = lane + 64 * q;
    if (i < body) dw[i] = __builtin_amdgcn_alignbit(hi[q], lo[q], 8 * head);
  }
  const int done = head + 4 * body;
  if (lane < NB - done) {
    const int b = done + lane;
    dst[b] = (uint8_t)(src[b >> 2] >> (8 * (b & 3)));
  }
}

// PAD = false runs every NTT / INTT transpose of the kernel on the unpadded
// (bank-conflicted) LDS layout: the padding step of the optimisation ablation.
// sched = hmax | tail << 8: hmax (1..G) tasks a workgroup holds at a time;
// with TAIL, tail slots per held task once the queue has run dry
// (sched_slots), else full batches of G slots (tail is then 0).  TAIL is a
// template switch so that the full-batch kernel keeps its register
// allocation (two wavefronts per SIMD with no spills at every level).
template <int LV, int NW, bool PAD = true, bool TAIL = false>
__global__ void __launch_bounds__(64 * NW) sg_persistw_k(Ws ws, PScr sc, uint8_t *sig, uint32_t count,
                                                     uint32_t sched, uint32_t *stats) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, G = PCfgW<LV, NW>::G, W = NW;
  constexpr bool CONTIG = NW == 4 && L == 4 && PAD;  // contiguous slot ranges per wavefront
  static_assert(G <= 64, "the winner search takes one slot per lane");
  static_assert(!CONTIG || PCfgW<LV, NW>::GW * L <= 64, "a wavefront's own slots take one ExpandMask lane per stream");
  __shared__ PersistWLds<LV, NW> lds;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, t = lane & 15;
  const size_t wg = blockIdx.x;
  const ScratchIdx si = scratch_idx<LV>(G);
  int32_t *yb = sc.y + si.y(wg, 0, 0);
  int32_t *wb = sc.w + si.w(wg, 0, 0);
  uint8_t *w1b = sc.w1 + si.w1(wg, 0);
  uint8_t *stg = sc.stage + si.stage(wg, 0);
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  if (tid == 0) {
    lds.tally.clear();
    lds.nheld = 0;
    lds.queue_empty = 0;
  }
  __syncthreads();
#ifdef DIL_PHASE_TIMERS
  uint64_t ph_t = __builtin_amdgcn_s_memtime();  // lane 0 of every wavefront times the barrier-separated phases
  uint64_t ph_acc[5] = {0, 0, 0, 0, 0};
#endif
  for (uint32_t batch = 0;; batch++) {
    if (tid == 0) {
      int nh = lds.nheld;
      const int hmax = (int)(sched & 0xFFu), tail = (int)(sched >> 8);
      if (!lds.queue_empty && nh < hmax) nh = claim_tasks(ws.counters, count, (uint32_t)(hmax - nh), nh, lds.h_task,
                                                          lds.h_next, lds.queue_empty);
      lds.nheld = nh;
      const int want = TAIL ? sched_slots(nh, G, W, lds.queue_empty, tail) : G;
      const int ns = CONTIG ? sched_assign_contig(nh, want, lds.h_next, lds.h_win, lds.s_h, lds.s_att)
                            : sched_assign(nh, want, lds.h_next, lds.h_win, lds.s_h, lds.s_att);
      lds.nslots = ns;
      lds.tally.evaluated += (uint64_t)ns;
    }
    __syncthreads();
    const int ns = lds.nslots;
    if (ns == 0) break;
    PHASE_MARK(0);
    // the slots this wave takes in the w and check phases: w, w + W, ...
    // (CONTIG: its own range [s_lo, s_hi))
    int s_lo = wave, s_hi = ns;
    if constexpr (CONTIG) sched_wave_range(ns, W, wave, s_lo, s_hi);
    constexpr int s_step = CONTIG ? 1 : W;
    if constexpr (CONTIG) {
      // ExpandMask of the wave's own slots, one lane per (slot, i); the y
      // rows it writes are read back by other lanes of the same wave only
      if (s_lo + lane / L < s_hi) {
        int s = s_lo + lane / L, i = lane % L;
        uint32_t task = lds.h_task[lds.s_h[s]];
        dev_expand_mask<LV>(ws.rhop + (size_t)task * 64, lds.s_att[s] * (uint32_t)L, i, yb + si.y(0, s, i));
      }
      wave_sync_global();
    } else {
      // ExpandMask: one thread per (slot, i)
      if (tid < ns * L) {
        int s = tid / L, i = tid % L;
        uint32_t task = lds.h_task[lds.s_h[s]];
        dev_expand_mask<LV>(ws.rhop + (size_t)task * 64, lds.s_att[s] * (uint32_t)L, i, yb + si.y(0, s, i));
      }
      __threadfence_block();
      __syncthreads();
    }
    PHASE_MARK(1);
    // w per slot
    for (int s = s_lo; s < s_hi; s += s_step) {
      uint32_t task = lds.h_task[lds.s_h[s]];
      dev_compute_w<LV, PAD, CONTIG>(yb + si.y(0, s, 0), ws.A + kix(ws, task) * K * L * N, wb + si.w(0, s, 0),
                        w1b + si.w1(0, s), lds.u[wave].wp.hat,
                        lds.u[wave].wp.tr + (lane >> 4) * NTT_LDS_GROUP, lds.u[wave].wp.w1buf, ftw, itw, lane);
      wave_sync();
    }
    __threadfence_block();
    __syncthreads();
    PHASE_MARK(2);
    // challenges, two lanes per slot: slots 0..31 on the batch's first
    // (rotating) wave, slots 32.. on the next one
    {
      const int s = (wave - (int)((wg + batch) % W) + W) % W * 32 + (lane >> 1);
      if (s < ns) {
        uint32_t task = lds.h_task[lds.s_h[s]];
        dev_challenge_pair<LV>(ws.muw1 + (size_t)task * muw1_stride<LV>(), w1b + si.w1(0, s), lane & 1,
                               lds.ct[s], lds.c[s], lds.bb[s]);
      }
    }
    __syncthreads();
    PHASE_MARK(3);
    // checks; a slot is skipped once a smaller nonce of its task has passed
    for (int s = s_lo; s < s_hi; s += s_step) {
      int h = lds.s_h[s];
      // another wave may lower h_win meanwhile: read it once, wave-uniformly
      if (__builtin_amdgcn_readfirstlane(lds.h_win[h]) < lds.s_att[s]) continue;
      uint32_t task = lds.h_task[h];
      bool ok = dev_check<LV, PAD, CONTIG>(lds.c[s], lds.ct[s], yb + si.y(0, s, 0), wb + si.w(0, s, 0),
                              ws.s1h + kix(ws, task) * L * N, ws.s2h + kix(ws, task) * K * N,
                              ws.t0h + kix(ws, task) * K * N, lds.u[wave].ck, ftw, itw, lane);
      if (ok) {
        const uint32_t *sb = lds.u[wave].ck.sigbuf;
        uint32_t *dst = (uint32_t *)(stg + si.stage(0, s));
        for (int w = lane; w < (P<LV>::SIG + 3) / 4; w += 64) dst[w] = sb[w];
        if (lane == 0) atomicMin(&lds.h_win[h], lds.s_att[s]);
      }
      wave_sync();
    }
    __threadfence_block();
    __syncthreads();
    PHASE_MARK(4);
    // copy each signed task's smallest passing candidate out; wave w handles held tasks w, w + 4, ...
    for (int h = wave; h < lds.nheld; h += W) {
      const uint32_t win = lds.h_win[h];
      if (win == SCHED_NONE) continue;
      // the slot that evaluated the winning nonce, found by one ballot over
      // all slots (G <= 64); h_win only ever takes a slot's s_att, so it exists
      const uint64_t hit = __ballot(lane < ns && lds.s_h[lane] == h && lds.s_att[lane] == win);
      if (hit == 0) continue;
      const int s = (int)__builtin_ctzll(hit);
      copy_sig_row<P<LV>::SIG>((const uint32_t *)(stg + si.stage(0, s)),
                               sig + (size_t)lds.h_task[h] * P<LV>::SIG, lane);
    }
    __syncthreads();
    if (tid == 0)
      lds.nheld = sched_retire(lds.nheld, lds.h_task, lds.h_next, lds.h_win, (uint32_t)PCfg<LV>::MAX_ATTEMPTS,
                               lds.tally.sequential, lds.tally.dropped);
    __syncthreads();
  }
  if (tid == 0) lds.tally.flush(stats);
  PHASE_FLUSH();
}

}  // namespace dil
