// Persistent fused Sign kernel with a device-side work queue (Alg. 2 loop).
//
// The paper's host scheduler (Sec. 4.3) refills idle execution units between
// kernel rounds and predicts nonces for unfinished tasks, keeping the valid
// signature with the smallest nonce.  Here the whole rejection loop runs in
// one launch: each wavefront (one 64-lane workgroup) claims tasks from a
// global atomic counter and owns them until they are signed.  Per batch it
// evaluates G candidate iterations ("slots"); when it holds fewer than G
// tasks, the spare slots evaluate later iterations kappa + l*m of the same
// tasks.  Iterations of one task are assigned in increasing order and every
// earlier iteration has already failed, so the smallest passing kappa of the
// batch is the sequential algorithm's answer and is written straight to the
// task's signature row.  Stages run back to back inside the batch:
//   ExpandMask (one lane per stream) -> w = A y per slot (4 groups) ->
//   ctilde and SampleInBall (one lane per slot) -> checks per slot.
#pragma once
#include "kernels.h"

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
};

template <int LV>
__device__ __forceinline__ size_t w1_stride() {
  return ((size_t)Lv<LV>::K * P<LV>::W1B + 255) & ~(size_t)255;
}

// Optional per-phase cycle accounting (compile with -DDIL_PHASE_TIMERS): lane 0 of
// every workgroup adds the s_memtime cycles of each batch phase to stats[8 + p].
#ifdef DIL_PHASE_TIMERS
#define PHASE_MARK(p)                                                              \
  do {                                                                             \
    uint64_t now_ = __builtin_amdgcn_s_memtime();                                  \
    if (lane == 0) atomicAdd((unsigned long long *)&stats[16 + 2 * (p)], now_ - ph_t); \
    ph_t = now_;                                                                   \
  } while (0)
#else
#define PHASE_MARK(p) \
  do {                \
  } while (0)
#endif

__device__ __forceinline__ void wave_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int LV>
struct PersistLds {
  union {
    struct {
      int32_t hat[Lv<LV>::L * N];
      int32_t tr[4 * NTT_LDS_GROUP];
      uint32_t w1buf[Lv<LV>::K * P<LV>::W1B / 4 + 1];
    } wp;
    CheckLds<LV> ck;
  } u;
  int8_t c[PCfg<LV>::G][N];
  uint32_t ct[PCfg<LV>::G][8];
  uint32_t bb[PCfg<LV>::G][RATE256 / 4];
  uint32_t h_task[PCfg<LV>::G], h_next[PCfg<LV>::G], h_win[PCfg<LV>::G];
  uint32_t s_att[PCfg<LV>::G];
  uint8_t s_h[PCfg<LV>::G];
  int nheld, nslots, queue_empty;
};

// ws.counters[0] is the work queue (next task to claim).  stats (32-bit words,
// zeroed by the host): [2..3] candidates evaluated (u64), [5] tasks dropped at
// MAX_ATTEMPTS, [6..7] sequential iterations = sum over tasks of (winning
// index + 1) (u64)
template <int LV>
__global__ void __launch_bounds__(64) sg_persist_k(Ws ws, PScr sc, uint8_t *sig, uint32_t count, uint32_t hmax,
                                                   uint32_t *stats) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L, G = PCfg<LV>::G;
  __shared__ PersistLds<LV> lds;
  const int lane = threadIdx.x, t = lane & 15;
  const size_t wg = blockIdx.x;
  int32_t *yb = sc.y + wg * G * L * N;
  int32_t *wb = sc.w + wg * G * K * N;
  uint8_t *w1b = sc.w1 + wg * G * w1_stride<LV>();
  const Tw ftw = ntt_lane_tw(t), itw = intt_lane_tw(t);
  if (lane == 0) {
    lds.nheld = 0;
    lds.queue_empty = 0;
  }
  wave_sync();
#ifdef DIL_PHASE_TIMERS
  uint64_t ph_t = __builtin_amdgcn_s_memtime();
#endif
  for (;;) {
    // ---- claim tasks and assign the batch's slots ----
    if (lane == 0) {
      int nh = lds.nheld;
      while (!lds.queue_empty && nh < (int)hmax) {
        uint32_t tk = atomicAdd(&ws.counters[0], 1u);
        if (tk >= count) {
          lds.queue_empty = 1;
          break;
        }
        lds.h_task[nh] = tk;
        lds.h_next[nh] = 0;
        nh++;
      }
      lds.nheld = nh;
      int ns = nh ? G : 0;
      for (int s = 0; s < ns; s++) {
        int h = s % nh;
        lds.s_h[s] = (uint8_t)h;
        lds.s_att[s] = lds.h_next[h] + (uint32_t)(s / nh);
      }
      for (int h = 0; h < nh; h++) {
        lds.h_next[h] += (uint32_t)(ns / nh + (h < ns % nh ? 1 : 0));
        lds.h_win[h] = 0xFFFFFFFFu;
      }
      lds.nslots = ns;
      if (ns) atomicAdd((unsigned long long *)&stats[2], (unsigned long long)ns);
    }
    wave_sync();
    const int ns = lds.nslots;
    if (ns == 0) break;
    PHASE_MARK(0);
    // ---- ExpandMask: one lane per (slot, i) ----
    if (lane < ns * L) {
      int s = lane / L, i = lane % L;
      uint32_t task = lds.h_task[lds.s_h[s]];
      dev_expand_mask<LV>(ws.rhop + (size_t)task * 64, lds.s_att[s] * (uint32_t)L, i, yb + ((size_t)s * L + i) * N);
    }
    wave_sync_global();
    PHASE_MARK(1);
    // ---- w = INTT(A NTT(y)) per slot ----
    for (int s = 0; s < ns; s++) {
      uint32_t task = lds.h_task[lds.s_h[s]];
      dev_compute_w<LV>(yb + (size_t)s * L * N, ws.A + kix(ws, task) * K * L * N, wb + (size_t)s * K * N,
                        w1b + s * w1_stride<LV>(), lds.u.wp.hat, lds.u.wp.tr + (lane >> 4) * NTT_LDS_GROUP,
                        lds.u.wp.w1buf, ftw, itw, lane);
      wave_sync();
    }
    wave_sync_global();
    PHASE_MARK(2);
    // ---- ctilde and SampleInBall: one lane per slot ----
    if (lane < ns) {
      uint32_t task = lds.h_task[lds.s_h[lane]];
      dev_challenge<LV>(ws.muw1 + (size_t)task * muw1_stride<LV>(), w1b + lane * w1_stride<LV>(), lds.ct[lane],
                        lds.c[lane], (uint8_t *)lds.bb[lane]);
    }
    wave_sync();
    PHASE_MARK(3);
    // ---- checks, in slot order; the first pass of a task is its signature ----
    for (int s = 0; s < ns; s++) {
      int h = lds.s_h[s];
      if (lds.h_win[h] != 0xFFFFFFFFu) continue;
      uint32_t task = lds.h_task[h];
      bool ok = dev_check<LV>(lds.c[s], lds.ct[s], yb + (size_t)s * L * N, wb + (size_t)s * K * N,
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
    if (lane == 0) {
      int nh = lds.nheld, o = 0;
      for (int h = 0; h < nh; h++) {
        if (lds.h_win[h] != 0xFFFFFFFFu) {
          atomicAdd((unsigned long long *)&stats[6], (unsigned long long)(lds.h_win[h] + 1));
          continue;
        }
        if (lds.h_next[h] >= (uint32_t)PCfg<LV>::MAX_ATTEMPTS) {
          atomicAdd(&stats[5], 1u);
          continue;
        }
        lds.h_task[o] = lds.h_task[h];
        lds.h_next[o] = lds.h_next[h];
        o++;
      }
      lds.nheld = o;
    }
    wave_sync();
  }
}

}  // namespace dil
