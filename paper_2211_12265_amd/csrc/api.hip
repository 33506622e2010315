// Host side of libdil: context, workspace pool and the C-ABI entry points.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/dil.h"
#include "errwords.h"
#include "ntt_ablation.h"
#include "t0_ablation.h"
#include "persist.h"
#include "probe.h"

using namespace dil;

// Scratch of the entry point that allocates nothing (dil_verify_keyset_noalloc);
// host code reaches it only through the per-device address from
// hipGetSymbolAddress (scratch_address below).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

struct dil_ctx {
  int device = 0;
  int mode = DIL_MODE_STAGED;
  void *ws_mem = nullptr;
  size_t ws_bytes = 0;
  uint32_t *host_counters = nullptr;  // pinned, 16 words
  char err[256] = {0};
  uint64_t stat_evaluated = 0, stat_sequential = 0;
  uint32_t *dev_stats = nullptr;      // 16 words: statistics of the last persistent Sign
  hipStream_t last_stream = nullptr;
  int stats_pending = 0;
  int64_t persist_grid = 0, persist_hmax = 0;  // 0 = automatic
  int persist_tail = -1;                       // slots per held task once the work queue is empty
                                               // (0 = all G; -1 = the level's default, PCfgW::TAIL_AUTO)
  int persist_waves = 4;                       // wavefronts per persistent workgroup: 1, 2 or 4
  int timing = 0;                              // record HIP events around the persistent Sign phases
  int ntt_variant = 0;                         // form of dil_ntt_mul_batch (0 = production kernel)
  int t0_variant = 0;                          // form of dil_t0_ntt_batch (0 = production code path)
  int persist_pad = 1;                         // 0: four-wavefront loop kernel on unpadded LDS transposes
  int mldsa_internal = 0;                      // 1: ML-DSA messages are formatted messages M' (mu = H(tr || M'))
  static constexpr int RING = 64;
  hipEvent_t ev[RING][3] = {};                 // per timed call: before setup, before loop, after loop
  int ev_count = 0;                            // timed calls recorded since timing was (re)enabled
  int cu_count = 0;                            // cached device properties
  int occ[4][6] = {};                          // cached persistent-kernel occupancy [1/2/4 waves, 4 with tail][lv_slot]
  // hipGraph replay of identical calls (same level, buffers, count and schedule)
  int use_graph = 0;
  hipStream_t cap_stream = nullptr;            // private stream the graphs are captured on
  struct Graph {
    uint64_t key[16];
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  std::vector<Graph> graphs;
  uint64_t clock = 0;
  int graph_hits = 0, graph_builds = 0;
  // side streams for independent setup stages (fork/join through events)
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
  hipEvent_t done_ev = nullptr;                // recorded after each call's last enqueue
  uint8_t *scratch = nullptr;                  // this device's no-alloc scratch array (device address)
  int pool_alloc = 0;                          // workspace from the stream-ordered allocator
};

struct dil_keyset {
  int level = 0;
  uint32_t nkeys = 0;
  int device = 0;
  void *mem = nullptr;
  uint8_t *pk = nullptr, *sk = nullptr, *tr = nullptr;   // key rows (copies) and tr = H(pk)
  size_t bytes = 0;                                      // device memory held
  int32_t *A = nullptr, *s1h = nullptr, *s2h = nullptr, *t0h = nullptr, *t1h = nullptr;
};

namespace {

int fail(dil_ctx *ctx, int code, const char *what, hipError_t e = hipSuccess) {
  if (ctx) {
    if (e != hipSuccess) snprintf(ctx->err, sizeof ctx->err, "%s: %s", what, hipGetErrorString(e));
    else snprintf(ctx->err, sizeof ctx->err, "%s", what);
  }
  return code;
}

#define HIPCHK(ctx, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return fail(ctx, DIL_EHIP, #call, e_); \
  } while (0)

#define LAUNCHCHK(ctx)                                     \
  do {                                                     \
    hipError_t e_ = hipGetLastError();                     \
    if (e_ != hipSuccess) return fail(ctx, DIL_EHIP, "kernel launch", e_); \
  } while (0)

void drop_graphs(dil_ctx *ctx) {
  for (auto &g : ctx->graphs) hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
}

// round-3 levels 2 / 3 / 5 (Tab. 1) and the ML-DSA-44 / 65 / 87 parameter sets of FIPS 204
bool valid_level(int lv) { return lv == 2 || lv == 3 || lv == 5 || lv == 44 || lv == 65 || lv == 87; }
bool mldsa_level(int lv) { return lv == 44 || lv == 65 || lv == 87; }
// Sign / Verify calls on formatted messages ("mldsa.internal") exist at the ML-DSA levels only
int check_form(dil_ctx *ctx, int level) {
  if (ctx->mldsa_internal && !mldsa_level(level))
    return fail(ctx, DIL_EINVAL, "mldsa.internal = 1 applies to the ML-DSA levels 44 / 65 / 87");
  return DIL_OK;
}
constexpr int lv_slot(int lv) { return lv == 2 ? 0 : lv == 3 ? 1 : lv == 5 ? 2 : lv == 44 ? 3 : lv == 65 ? 4 : 5; }

// The kinds of call a workspace is laid out for: each carves only the
// per-task rows its kernels read or write.
enum WsForm { WS_KEYGEN = 0, WS_SIGN_STAGED = 1, WS_SIGN_PERSIST = 2, WS_VERIFY = 3 };

template <int LV>
constexpr int persist_slots(int waves) {
  return waves == 1 ? PCfg<LV>::G : waves * PCfg<LV>::G;
}

// Lay out the workspace of a call of `cap` tasks at `base` (nullptr: only
// count) and return its size in bytes.  Every row is 256-byte aligned.  With a
// resident key table (keyset) A-hat and the NTT-domain secrets come from the
// table and are not carved; the persistent form adds its per-workgroup scratch
// for `grid` workgroups of `waves` wavefronts.
template <int LV>
size_t ws_layout(uint8_t *base, size_t cap, int form, bool keyset, size_t grid, int waves, Ws *ws, PScr *sc,
                 uint32_t **kidx) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  const bool sign = form == WS_SIGN_STAGED || form == WS_SIGN_PERSIST, staged = form == WS_SIGN_STAGED;
  size_t off = 0;
  auto take = [&](bool used, size_t bytes) -> uint8_t * {
    if (!used) return nullptr;
    uint8_t *r = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return r;
  };
  const size_t muw1_stride = ((size_t)P<LV>::MUW1 + 255) & ~(size_t)255;
  Ws w{};
  w.cap = cap;
  w.muw1_stride = muw1_stride;
  w.counters = (uint32_t *)take(true, 16 * 4);
  w.muw1 = take(sign || form == WS_VERIFY, cap * muw1_stride);
  w.rhop = take(sign || form == WS_KEYGEN, cap * 64);
  w.ctilde = take(staged, cap * CT_STRIDE);
  w.cpoly = (int8_t *)take(staged || form == WS_VERIFY, cap * 256);
  w.A = (int32_t *)take(!keyset, cap * K * L * 1024);
  w.s1h = (int32_t *)take(form == WS_KEYGEN || (sign && !keyset), cap * (form == WS_KEYGEN ? L + K : L) * 1024);
  w.s2h = (int32_t *)take(sign && !keyset, cap * K * 1024);
  w.t0h = (int32_t *)take(sign && !keyset, cap * K * 1024);
  w.y = (int32_t *)take(staged, cap * L * 1024);
  w.w = (int32_t *)take(staged, cap * K * 1024);
  w.hmask = (uint32_t *)take(form == WS_VERIFY, cap * K * 32);
  w.flag = (int32_t *)take(form == WS_VERIFY, cap * 4);
  w.kappa = (uint32_t *)take(sign, cap * 4);
  w.active0 = (uint32_t *)take(sign, cap * 4);
  w.active1 = (uint32_t *)take(staged, cap * 4);
  uint32_t *kid = (uint32_t *)take(keyset, cap * 4);  // checked key indices of key-table calls
  PScr p{};
  if (form == WS_SIGN_PERSIST) {
    // the regions the loop kernels index with the same ScratchIdx (batch_sched.h)
    const ScratchIdx si{(size_t)persist_slots<LV>(waves), (size_t)L, (size_t)K, w1_stride<LV>(), sig_stride<LV>()};
    p.y = (int32_t *)take(true, si.y_size(grid) * sizeof(int32_t));
    p.w = (int32_t *)take(true, si.w_size(grid) * sizeof(int32_t));
    p.w1 = take(true, si.w1_size(grid));
    p.stage = take(waves > 1, si.stage_size(grid));
  }
  if (ws) *ws = w;
  if (sc) *sc = p;
  if (kidx) *kidx = kid;
  return off;
}

// Record the end of a call's work on its stream: a later workspace growth
// waits for this event (the last call of the context) instead of the device.
int mark_done(dil_ctx *ctx, hipStream_t st) {
  if (!ctx->done_ev) HIPCHK(ctx, hipEventCreateWithFlags(&ctx->done_ev, hipEventDisableTiming));
  HIPCHK(ctx, hipEventRecord(ctx->done_ev, st));
  return DIL_OK;
}

// Make sure the context's workspace holds `need` bytes.  Growing it waits for
// the context's own last call (calls on one context are ordered by contract),
// drops the graphs that captured the old addresses and replaces the memory in
// stream order on `st`, so other contexts and streams never stall on it.
int ws_reserve_bytes(dil_ctx *ctx, size_t need, hipStream_t st) {
  if (need <= ctx->ws_bytes) return DIL_OK;
  if (ctx->done_ev) HIPCHK(ctx, hipEventSynchronize(ctx->done_ev));
  drop_graphs(ctx);
  if (ctx->ws_mem) {
    // (hipFree would synchronise the whole device)
    if (ctx->pool_alloc) HIPCHK(ctx, hipFreeAsync(ctx->ws_mem, st));
    else HIPCHK(ctx, hipFree(ctx->ws_mem));
    ctx->ws_mem = nullptr;
    ctx->ws_bytes = 0;
  }
  hipError_t e = ctx->pool_alloc ? hipMallocAsync(&ctx->ws_mem, need, st) : hipMalloc(&ctx->ws_mem, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws_mem = nullptr;
    return fail(ctx, DIL_ENOMEM, "workspace allocation", e);
  }
  ctx->ws_bytes = need;
  return DIL_OK;
}

template <int LV>
int ws_carve(dil_ctx *ctx, hipStream_t st, size_t cap, int form, bool keyset, Ws &ws, size_t grid = 0,
             PScr *sc = nullptr, int waves = 1, uint32_t **kidx = nullptr) {
  const size_t need = ws_layout<LV>(nullptr, cap, form, keyset, grid, waves, nullptr, nullptr, nullptr);
  int rc = ws_reserve_bytes(ctx, need, st);
  if (rc) return rc;
  const size_t got = ws_layout<LV>((uint8_t *)ctx->ws_mem, cap, form, keyset, grid, waves, &ws, sc, kidx);
  if (got > ctx->ws_bytes) return fail(ctx, DIL_ENOMEM, "workspace layout overflow");
  ws.kmap = nullptr;
  ws.t1h = nullptr;
  ws.tr = nullptr;
  return DIL_OK;
}

// Read and clear the device-detected error words (errwords.h) after the work
// enqueued on `st`; synchronises `st`.
int take_msg_error(dil_ctx *ctx, hipStream_t st) {
  HIPCHK(ctx, hipMemcpyAsync(ctx->host_counters, ctx->dev_stats, 16 * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  const uint32_t dropped = ctx->host_counters[ERR_WORD_DROPPED], msg_flag = ctx->host_counters[ERR_WORD_MSG],
                 key_flag = ctx->host_counters[ERR_WORD_KEY];
  char text[sizeof ctx->err];
  const int code = report_error_words(dropped, msg_flag, key_flag, text, sizeof text);
  if (code == DIL_OK) return DIL_OK;
  zero_words_k<<<1, 64, 0, st>>>(ctx->dev_stats + ERR_WORD_DROPPED, 1, ctx->dev_stats + ERR_WORD_MSG, 2);
  LAUNCHCHK(ctx);
  HIPCHK(ctx, hipStreamSynchronize(st));
  return fail(ctx, code, text);
}

// Enqueue fn(stream) on st, or -- with graphs enabled -- replay the graph that
// captured fn for this exact key (capturing it on first use).
template <class F>
int enqueue(dil_ctx *ctx, const uint64_t *key, hipStream_t st, F fn) {
  if (!ctx->use_graph) return fn(st);
  ctx->clock++;
  for (auto &g : ctx->graphs)
    if (!memcmp(g.key, key, sizeof g.key)) {
      g.last_use = ctx->clock;
      ctx->graph_hits++;
      HIPCHK(ctx, hipGraphLaunch(g.exec, st));
      return DIL_OK;
    }
  if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
  int rc = fn(ctx->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (rc) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(ctx, DIL_EHIP, "graph capture", e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ctx, DIL_EHIP, "graph instantiate", e);
  if (ctx->graphs.size() >= 16) {  // evict the least recently used
    auto it = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                               [](const dil_ctx::Graph &x, const dil_ctx::Graph &y) { return x.last_use < y.last_use; });
    hipGraphExecDestroy(it->exec);
    ctx->graphs.erase(it);
  }
  dil_ctx::Graph g;
  memcpy(g.key, key, sizeof g.key);
  g.exec = exec;
  g.last_use = ctx->clock;
  ctx->graphs.push_back(g);
  ctx->graph_builds++;
  HIPCHK(ctx, hipGraphLaunch(exec, st));
  return DIL_OK;
}

// Fork: side streams wait for everything enqueued on st so far.
int fork_side(dil_ctx *ctx, hipStream_t st) {
  if (!ctx->side[0]) {
    for (int i = 0; i < 2; i++) {
      HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
      HIPCHK(ctx, hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming));
    }
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming));
  }
  HIPCHK(ctx, hipEventRecord(ctx->fork_ev, st));
  for (int i = 0; i < 2; i++) HIPCHK(ctx, hipStreamWaitEvent(ctx->side[i], ctx->fork_ev, 0));
  return DIL_OK;
}
// Join: st waits for the work enqueued so far on side stream i.
int join_one(dil_ctx *ctx, hipStream_t st, int i) {
  HIPCHK(ctx, hipEventRecord(ctx->join_ev[i], ctx->side[i]));
  HIPCHK(ctx, hipStreamWaitEvent(st, ctx->join_ev[i], 0));
  return DIL_OK;
}
// Join: st waits for both side streams' work.
int join_side(dil_ctx *ctx, hipStream_t st) {
  for (int i = 0; i < 2; i++) {
    int rc = join_one(ctx, st, i);
    if (rc) return rc;
  }
  return DIL_OK;
}

inline unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

template <int LV>
int keygen_impl(dil_ctx *ctx, const uint8_t *seeds, uint8_t *pk, uint8_t *sk, uint32_t count, hipStream_t st) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  Ws ws;
  int rc = ws_carve<LV>(ctx, st, count, WS_KEYGEN, false, ws);
  if (rc) return rc;
  kg_seed_k<LV><<<blocks_for(count, 256), 256, 0, st>>>(seeds, pk, sk, ws, count);
  expand_a_k<LV><<<blocks_for((uint64_t)count * K * L, EA_WG), EA_WG, 0, st>>>(pk, P<LV>::PK, nullptr, ws.A, count);
  expand_s_k<LV><<<blocks_for((uint64_t)count * (K + L), 256), 256, 0, st>>>(ws, count);
  kg_main_k<LV><<<count, 64, 0, st>>>(ws, pk, sk, count);
  kg_tr_k<LV><<<blocks_for(count, 256), 256, 0, st>>>(pk, sk, count);
  LAUNCHCHK(ctx);
  return mark_done(ctx, st);
}

// Resident key tables replace the per-task A-hat / NTT(s) arrays (no ExpandA,
// no secret NTTs).  A caller's key_idx is read only once, by keys_check_k
// (check_keys below), which writes a copy with every index inside the table
// to `checked`; every other kernel of the call reads that copy, which this
// returns (nullptr when the call has no key_idx: task i uses row i).
const uint32_t *use_keyset(Ws &ws, const dil_keyset *ks, const uint32_t *key_idx, uint32_t *checked) {
  ws.A = ks->A;
  ws.s1h = ks->s1h;
  ws.s2h = ks->s2h;
  ws.t0h = ks->t0h;
  ws.t1h = ks->t1h;
  ws.tr = ks->tr;
  ws.kmap = key_idx ? checked : nullptr;
  return ws.kmap;
}
void check_keys(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, uint32_t *checked, uint32_t count,
                hipStream_t st) {
  if (ks && key_idx)
    keys_check_k<<<blocks_for(count, 256), 256, 0, st>>>(key_idx, ks->nkeys, checked, count, ctx->dev_stats + 9);
}

// The setup stages are independent of each other: mu/rho' hash chains (one lane
// per task, latency-bound for small batches), ExpandA (one lane per stream) and
// the secret NTTs (one wave per task).  With `concurrent` they run on the
// context's side streams so the long chains overlap the bulk work.
template <int LV>
int sign_setup(dil_ctx *ctx, Ws &ws, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
               const uint64_t *msg_off, uint32_t count, hipStream_t st, const dil_keyset *ks, uint32_t *err,
               bool concurrent, const uint8_t *rnd) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  concurrent = concurrent && !ks;
  if (concurrent) {
    int rc = fork_side(ctx, st);
    if (rc) return rc;
  }
  const unsigned nb = blocks_for(2 * (uint64_t)count, 256);
  bool internal = false;
  if constexpr (Lv<LV>::MLDSA) internal = ctx->mldsa_internal;
  if constexpr (Lv<LV>::MLDSA) {
    if (internal) sg_prep_k<LV, true><<<nb, 256, 0, st>>>(sk, key_idx, msg, msg_off, rnd, ws, count, err);
  }
  if (!internal) sg_prep_k<LV><<<nb, 256, 0, st>>>(sk, key_idx, msg, msg_off, rnd, ws, count, err);
  if (!ks) {
    hipStream_t s1 = concurrent ? ctx->side[0] : st, s2 = concurrent ? ctx->side[1] : st;
    expand_a_k<LV><<<blocks_for((uint64_t)count * K * L, EA_WG), EA_WG, 0, s1>>>(sk, P<LV>::SK, key_idx, ws.A, count);
    sg_secret_k<LV><<<count, 64, 0, s2>>>(sk, key_idx, ws, count);
  }
  if (concurrent) return join_side(ctx, st);
  return DIL_OK;
}

template <int LV>
int sign_staged(dil_ctx *ctx, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg, const uint64_t *msg_off,
                uint8_t *sig, uint32_t count, hipStream_t st, const dil_keyset *ks = nullptr,
                const uint8_t *rnd = nullptr) {
  constexpr int L = Lv<LV>::L;
  Ws ws;
  uint32_t *kid = nullptr;
  int rc = ws_carve<LV>(ctx, st, count, WS_SIGN_STAGED, ks != nullptr, ws, 0, nullptr, 1, &kid);
  if (rc) return rc;
  if (ks) {
    check_keys(ctx, ks, key_idx, kid, count, st);
    key_idx = use_keyset(ws, ks, key_idx, kid);
  }
  HIPCHK(ctx, hipMemsetAsync(ws.counters, 0, 16 * 4, st));
  rc = sign_setup<LV>(ctx, ws, sk, key_idx, msg, msg_off, count, st, ks, ctx->dev_stats + 8, false, rnd);
  if (rc) return rc;
  LAUNCHCHK(ctx);
  uint32_t nactive = count;
  uint32_t *cur = ws.active0, *nxt = ws.active1;
  uint64_t evaluated = 0;
  int rounds = 0;
  while (nactive > 0) {
    if (++rounds > 4096) return fail(ctx, DIL_EHIP, "sign loop did not terminate");
    evaluated += nactive;
    HIPCHK(ctx, hipMemsetAsync(ws.counters, 0, 4, st));
    expand_mask_k<LV><<<blocks_for((uint64_t)nactive * L, 256), 256, 0, st>>>(ws, cur, nactive);
    sg_w_k<LV><<<nactive, 64, 0, st>>>(ws, cur, nactive);
    sg_chal_k<LV><<<blocks_for(nactive, 64), 64, 0, st>>>(ws, cur, nactive);
    sg_check_k<LV><<<nactive, 64, 0, st>>>(ws, sig, cur, nactive, nxt);
    LAUNCHCHK(ctx);
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_counters, ws.counters, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    nactive = ctx->host_counters[0];
    std::swap(cur, nxt);
  }
  ctx->stat_evaluated = evaluated;
  ctx->stat_sequential = evaluated;
  rc = mark_done(ctx, st);
  if (rc) return rc;
  return take_msg_error(ctx, st);
}

// Tail slots per held task of the context's persistent Sign calls at level LV
// ("persist.tail"; -1 = the level's default for the four-wavefront padded
// kernel, full batches for the other shapes).
template <int LV>
int tail_slots(const dil_ctx *ctx) {
  if (ctx->persist_tail >= 0) return ctx->persist_tail;
  return ctx->persist_waves == 4 && ctx->persist_pad ? PCfgW<LV, 4>::TAIL_AUTO : 0;
}

// resident workgroups per CU of the persistent kernel the context's shape launches (cached)
template <int LV>
int persist_occupancy(dil_ctx *ctx, int *occ) {
  if (!ctx->cu_count) {
    hipDeviceProp_t prop;
    HIPCHK(ctx, hipGetDeviceProperties(&prop, ctx->device));
    ctx->cu_count = prop.multiProcessorCount;
  }
  const int w = ctx->persist_waves;
  const bool tail = w == 4 && tail_slots<LV>(ctx) > 0;
  const int si = tail ? 3 : w == 4 ? 2 : w == 2 ? 1 : 0;
  if (Lv<LV>::MLDSA && w != 4) return fail(ctx, DIL_EINVAL, "ML-DSA levels run the four-wavefront loop kernel only");
  int &o = ctx->occ[si][lv_slot(LV)];
  if (!o) {
    if (tail) {
      HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sg_persistw_k<LV, 4, true, true>, 256, 0));
    } else if (w == 4) {
      HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sg_persistw_k<LV, 4>, 256, 0));
    } else if constexpr (!Lv<LV>::MLDSA) {
      if (w == 2) HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sg_persistw_k<LV, 2>, 128, 0));
      else HIPCHK(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sg_persist_k<LV>, 64, 0));
    }
  }
  *occ = std::max(o, 1);
  return DIL_OK;
}

// Schedule of a persistent Sign call of `count` tasks: workgroups launched and
// tasks each holds at a time (the "persist.*" knobs, else one wave of
// resident workgroups sharing the tasks evenly).
template <int LV>
int persist_schedule(dil_ctx *ctx, uint32_t count, uint64_t *grid_out, uint64_t *hmax_out) {
  const int G = persist_slots<LV>(ctx->persist_waves);
  int occ = 1;
  int rc = persist_occupancy<LV>(ctx, &occ);
  if (rc) return rc;
  const uint64_t pmax = (uint64_t)occ * ctx->cu_count, n = std::max<uint32_t>(count, 1);
  uint64_t hmax = ctx->persist_hmax > 0 ? (uint64_t)ctx->persist_hmax : (n + pmax - 1) / pmax;
  hmax = std::min<uint64_t>(std::max<uint64_t>(hmax, 1), G);
  uint64_t grid = ctx->persist_grid > 0 ? (uint64_t)ctx->persist_grid : std::min<uint64_t>(pmax, (n + hmax - 1) / hmax);
  *grid_out = std::max<uint64_t>(grid, 1);
  *hmax_out = hmax;
  return DIL_OK;
}

template <int LV>
int sign_persistent(dil_ctx *ctx, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                    const uint64_t *msg_off, uint8_t *sig, uint32_t count, hipStream_t st,
                    const dil_keyset *ks = nullptr, const uint8_t *rnd = nullptr) {
  const int waves = ctx->persist_waves;
  if (!ctx->persist_pad && waves != 4)
    return fail(ctx, DIL_EINVAL, "persist.pad = 0 exists for the four-wavefront loop kernel only");
  // the one- and two-wavefront shapes and the unpadded ablation form are built for the round-3 levels only
  if (Lv<LV>::MLDSA && (waves != 4 || !ctx->persist_pad))
    return fail(ctx, DIL_EINVAL, "ML-DSA levels run the four-wavefront padded loop kernel (persist.waves = 4, persist.pad = 1)");
  if (ctx->persist_tail > 0 && (waves != 4 || !ctx->persist_pad))
    return fail(ctx, DIL_EINVAL, "persist.tail > 0 exists for the four-wavefront padded loop kernel only");
  const int ntail = tail_slots<LV>(ctx);
  uint64_t grid = 1, hmax = 1;
  int rc = persist_schedule<LV>(ctx, count, &grid, &hmax);
  if (rc) return rc;
  Ws ws;
  PScr sc;
  uint32_t *kid = nullptr;
  rc = ws_carve<LV>(ctx, st, count, WS_SIGN_PERSIST, ks != nullptr, ws, grid, &sc, waves, &kid);
  if (rc) return rc;
  const uint32_t *key_in = key_idx;
  if (ks) key_idx = use_keyset(ws, ks, key_idx, kid);
  uint64_t key[16] = {1, (uint64_t)LV, (uint64_t)sk, (uint64_t)key_in, (uint64_t)msg, (uint64_t)msg_off,
                      (uint64_t)sig, count, (uint64_t)ks, grid, hmax, (uint64_t)ctx->ws_mem, 0, (uint64_t)waves,
                      (uint64_t)rnd, (uint64_t)ctx->mldsa_internal};
  hipEvent_t *evs = ctx->timing ? ctx->ev[ctx->ev_count % dil_ctx::RING] : nullptr;
  if (evs) HIPCHK(ctx, hipEventRecord(evs[0], st));
  rc = enqueue(ctx, key, st, [&](hipStream_t s) {
    zero_words_k<<<1, 64, 0, s>>>(ws.counters, 16, ctx->dev_stats, 8);
    check_keys(ctx, ks, key_in, kid, count, s);
    int r2 = sign_setup<LV>(ctx, ws, sk, key_idx, msg, msg_off, count, s, ks, ctx->dev_stats + 8, true, rnd);
    if (r2) return r2;
    LAUNCHCHK(ctx);
    return DIL_OK;
  });
  if (rc) return rc;
  if (evs) HIPCHK(ctx, hipEventRecord(evs[1], st));
  // The loop kernel is one launch: it is launched directly, also when graphs
  // are enabled (as a graph node it measured 2-4% slower).
  const bool tail = ntail > 0;
  const uint32_t sched = (uint32_t)hmax | (uint32_t)ntail << 8;  // hmax <= G <= 64, tail <= 64
  if constexpr (Lv<LV>::MLDSA) {
    if (tail) sg_persistw_k<LV, 4, true, true><<<(unsigned)grid, 256, 0, st>>>(ws, sc, sig, count, sched, ctx->dev_stats);
    else sg_persistw_k<LV, 4><<<(unsigned)grid, 256, 0, st>>>(ws, sc, sig, count, sched, ctx->dev_stats);
  } else {
    if (waves == 4 && !ctx->persist_pad)
      sg_persistw_k<LV, 4, false><<<(unsigned)grid, 256, 0, st>>>(ws, sc, sig, count, sched, ctx->dev_stats);
    else if (waves == 4 && tail)
      sg_persistw_k<LV, 4, true, true><<<(unsigned)grid, 256, 0, st>>>(ws, sc, sig, count, sched, ctx->dev_stats);
    else if (waves == 4)
      sg_persistw_k<LV, 4><<<(unsigned)grid, 256, 0, st>>>(ws, sc, sig, count, sched, ctx->dev_stats);
    else if (waves == 2)
      sg_persistw_k<LV, 2><<<(unsigned)grid, 128, 0, st>>>(ws, sc, sig, count, sched, ctx->dev_stats);
    else
      sg_persist_k<LV><<<(unsigned)grid, 64, 0, st>>>(ws, sc, sig, count, (uint32_t)hmax, ctx->dev_stats);
  }
  LAUNCHCHK(ctx);
  if (evs) {
    HIPCHK(ctx, hipEventRecord(evs[2], st));
    ctx->ev_count++;
  }
  ctx->last_stream = st;
  ctx->stats_pending = 1;
  return mark_done(ctx, st);
}

// Verify's tr / mu kernel in the context's message form
template <int LV>
void launch_vf_hash(const dil_ctx *ctx, hipStream_t st, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                    const uint64_t *msg_off, const Ws &ws, uint32_t count, uint32_t *err) {
  const unsigned nb = blocks_for(2 * (uint64_t)count, 64);
  if constexpr (Lv<LV>::MLDSA) {
    if (ctx->mldsa_internal) {
      vf_hash_k<LV, true><<<nb, 64, 0, st>>>(pk, key_idx, msg, msg_off, ws, count, err);
      return;
    }
  }
  vf_hash_k<LV><<<nb, 64, 0, st>>>(pk, key_idx, msg, msg_off, ws, count, err);
}

template <int LV>
int verify_impl(dil_ctx *ctx, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg, const uint64_t *msg_off,
                const uint8_t *sig, int32_t *verdict, uint32_t count, hipStream_t st,
                const dil_keyset *ks = nullptr) {
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  Ws ws;
  uint32_t *kid = nullptr;
  int rc = ws_carve<LV>(ctx, st, count, WS_VERIFY, ks != nullptr, ws, 0, nullptr, 1, &kid);
  if (rc) return rc;
  const uint32_t *key_in = key_idx;
  if (ks) key_idx = use_keyset(ws, ks, key_idx, kid);
  uint64_t key[16] = {2, (uint64_t)LV, (uint64_t)pk, (uint64_t)key_in, (uint64_t)msg, (uint64_t)msg_off,
                      (uint64_t)sig, (uint64_t)verdict, count, (uint64_t)ks, (uint64_t)ctx->ws_mem, 0, 0, 0, 0,
                      (uint64_t)ctx->mldsa_internal};
  rc = enqueue(ctx, key, st, [&](hipStream_t s) {
    zero_words_k<<<1, 64, 0, s>>>(ws.counters, 16, nullptr, 0);
    check_keys(ctx, ks, key_in, kid, count, s);
    // Three independent fronts: the tr / mu hash chain (needed only by the
    // final hash), ExpandA, and SampleInBall + hint decoding.  Outside the
    // staged form the first two run on side streams and are joined where
    // their results are first read.  With a resident key table there is no
    // ExpandA and tr is stored, so the calls (typically many small ones from
    // a serving loop) stay on one stream.
    const bool conc = ctx->mode != DIL_MODE_STAGED && !ks;
    if (conc) {
      int r2 = fork_side(ctx, s);
      if (r2) return r2;
    }
    hipStream_t s_hash = conc ? ctx->side[1] : s, s_ea = conc ? ctx->side[0] : s;
    launch_vf_hash<LV>(ctx, s_hash, pk, key_idx, msg, msg_off, ws, count, ctx->dev_stats + 8);
    if (!ks)
      expand_a_k<LV><<<blocks_for((uint64_t)count * K * L, EA_WG), EA_WG, 0, s_ea>>>(pk, P<LV>::PK, key_idx, ws.A,
                                                                                count);
    vf_prep_k<LV><<<blocks_for(count, 64), 64, 0, s>>>(sig, ws, count);
    if (conc) {
      int r2 = join_one(ctx, s, 0);
      if (r2) return r2;
    }
    vf_main_k<LV><<<count, 64, 0, s>>>(pk, key_idx, sig, ws, count);
    if (conc) {
      int r2 = join_one(ctx, s, 1);
      if (r2) return r2;
    }
    vf_final_k<LV><<<blocks_for(2 * (uint64_t)count, 256), 256, 0, s>>>(sig, ws, verdict, count);
    LAUNCHCHK(ctx);
    return DIL_OK;
  });
  if (rc) return rc;
  return mark_done(ctx, st);
}

template <int LV>
int keyset_build(dil_ctx *ctx, dil_keyset *ks, const uint8_t *pk, const uint8_t *sk, hipStream_t st) {
  using PP = P<LV>;
  constexpr int K = Lv<LV>::K, L = Lv<LV>::L;
  size_t n = ks->nkeys;
  size_t bytes = 0;
  auto rnd = [](size_t b) { return (b + 255) & ~(size_t)255; };
  bytes += rnd(n * K * L * 1024);
  if (sk) bytes += rnd(n * PP::SK) + rnd(n * L * 1024) + 2 * rnd(n * K * 1024);
  if (pk) bytes += rnd(n * PP::PK) + rnd(n * K * 1024);
  bytes += rnd(n * PP::TRB);
  hipError_t e = hipMalloc(&ks->mem, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, DIL_ENOMEM, "key table allocation", e);
  }
  ks->bytes = bytes;
  uint8_t *p = (uint8_t *)ks->mem;
  auto take = [&](size_t b) {
    uint8_t *r = p;
    p += rnd(b);
    return r;
  };
  ks->A = (int32_t *)take(n * K * L * 1024);
  ks->tr = take(n * PP::TRB);
  if (sk) {
    ks->sk = take(n * PP::SK);
    ks->s1h = (int32_t *)take(n * L * 1024);
    ks->s2h = (int32_t *)take(n * K * 1024);
    ks->t0h = (int32_t *)take(n * K * 1024);
    HIPCHK(ctx, hipMemcpyAsync(ks->sk, sk, n * PP::SK, hipMemcpyDeviceToDevice, st));
  }
  if (pk) {
    ks->pk = take(n * PP::PK);
    ks->t1h = (int32_t *)take(n * K * 1024);
    HIPCHK(ctx, hipMemcpyAsync(ks->pk, pk, n * PP::PK, hipMemcpyDeviceToDevice, st));
  }
  unsigned nb = blocks_for(n * K * L, EA_WG);
  if (sk) {
    expand_a_k<LV><<<nb, EA_WG, 0, st>>>(ks->sk, PP::SK, nullptr, ks->A, ks->nkeys);
    Ws w{};
    w.s1h = ks->s1h;
    w.s2h = ks->s2h;
    w.t0h = ks->t0h;
    sg_secret_k<LV><<<ks->nkeys, 64, 0, st>>>(ks->sk, nullptr, w, ks->nkeys);
  } else {
    expand_a_k<LV><<<nb, EA_WG, 0, st>>>(ks->pk, PP::PK, nullptr, ks->A, ks->nkeys);
  }
  if (pk) {
    ks_pk_k<LV><<<ks->nkeys, 64, 0, st>>>(ks->pk, ks->t1h, ks->nkeys);
    ks_tr_k<LV><<<blocks_for(n, 256), 256, 0, st>>>(ks->pk, ks->tr, ks->nkeys);
  } else {
    HIPCHK(ctx, hipMemcpy2DAsync(ks->tr, PP::TRB, ks->sk + 64, PP::SK, PP::TRB, n, hipMemcpyDeviceToDevice, st));
  }
  LAUNCHCHK(ctx);
  return DIL_OK;
}

// ---- scratch for the entry point that allocates nothing ----
// Device memory of dil_verify_keyset_noalloc: a file-scope device array (each
// GPU the library runs on holds its own copy until the process ends).  Host
// code never uses the array's name as an address: its device address is taken
// once per device with hipGetSymbolAddress (at context creation) and kept in
// scratch_ptr.  Every call on a GPU shares that GPU's copy; calls that
// overlap on one GPU race on it.
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on `device` (the current device).
int scratch_address(dil_ctx *ctx, int device, uint8_t **out) {
  if (device < 0 || device >= MAX_DEVICES) return fail(ctx, DIL_EINVAL, "device index above the scratch table");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(ctx, DIL_EHIP, "scratch address (hipGetSymbolAddress)", e);
    }
    scratch_ptr[device] = p;
  }
  *out = (uint8_t *)scratch_ptr[device];
  return DIL_OK;
}

template <class F>
int by_round3_level(int level, F f) {
  switch (level) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 5: return f(std::integral_constant<int, 5>{});
  }
  return DIL_EINVAL;
}
template <class F>
int by_level(int level, F f) {
  switch (level) {
    case 44: return f(std::integral_constant<int, 44>{});
    case 65: return f(std::integral_constant<int, 65>{});
    case 87: return f(std::integral_constant<int, 87>{});
  }
  return by_round3_level(level, f);
}

}  // namespace

extern "C" {

int dil_ctx_create(dil_ctx **out, int device, size_t workspace_bytes) {
  if (!out) return DIL_EINVAL;
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || device < 0 || device >= n) return DIL_EHIP;
  e = hipSetDevice(device);
  if (e != hipSuccess) return DIL_EHIP;
  dil_ctx *c = new dil_ctx();
  c->device = device;
  e = hipHostMalloc((void **)&c->host_counters, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return DIL_ENOMEM;
  }
  memset(c->host_counters, 0, 64);
  e = hipMalloc((void **)&c->dev_stats, 256);
  if (e == hipSuccess) {
    e = hipMemset(c->dev_stats, 0, 256);
    if (e != hipSuccess) hipFree(c->dev_stats);
  }
  if (e != hipSuccess) {
    hipHostFree(c->host_counters);
    delete c;
    return DIL_ENOMEM;
  }
  int pools = 0;
  c->pool_alloc = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device) == hipSuccess && pools;
  if (scratch_address(c, device, &c->scratch)) {
    dil_ctx_destroy(c);
    return DIL_EHIP;
  }
  if (workspace_bytes && (ws_reserve_bytes(c, workspace_bytes, nullptr) || hipStreamSynchronize(nullptr) != hipSuccess)) {
    dil_ctx_destroy(c);
    return DIL_ENOMEM;
  }
  *out = c;
  return DIL_OK;
}

int dil_ctx_destroy(dil_ctx *ctx) {
  if (!ctx) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->ws_mem) {
    if (ctx->pool_alloc) {
      hipFreeAsync(ctx->ws_mem, nullptr);
      hipStreamSynchronize(nullptr);
    } else {
      hipFree(ctx->ws_mem);
    }
  }
  if (ctx->done_ev) hipEventDestroy(ctx->done_ev);
  if (ctx->host_counters) hipHostFree(ctx->host_counters);
  if (ctx->dev_stats) hipFree(ctx->dev_stats);
  drop_graphs(ctx);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  for (int i = 0; i < 2; i++) {
    if (ctx->side[i]) hipStreamDestroy(ctx->side[i]);
    if (ctx->join_ev[i]) hipEventDestroy(ctx->join_ev[i]);
  }
  if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
  for (int r = 0; r < dil_ctx::RING; r++)
    for (int i = 0; i < 3; i++)
      if (ctx->ev[r][i]) hipEventDestroy(ctx->ev[r][i]);
  delete ctx;
  return DIL_OK;
}

int dil_ctx_set_mode(dil_ctx *ctx, int mode) {
  if (!ctx) return DIL_EINVAL;
  if (mode != DIL_MODE_STAGED && mode != DIL_MODE_PERSISTENT) return fail(ctx, DIL_EINVAL, "unsupported mode");
  ctx->mode = mode;
  return DIL_OK;
}

int dil_ctx_check(dil_ctx *ctx, void *stream) {
  if (!ctx) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  return take_msg_error(ctx, (hipStream_t)stream);
}

const char *dil_last_error(dil_ctx *ctx) { return ctx ? ctx->err : "null context"; }

int dil_ctx_set_param(dil_ctx *ctx, const char *name, int64_t value) {
  if (!ctx || !name) return DIL_EINVAL;
  if (!strcmp(name, "timing")) {
    if (value && !ctx->ev[0][0])
      for (int r = 0; r < dil_ctx::RING; r++)
        for (int i = 0; i < 3; i++) HIPCHK(ctx, hipEventCreate(&ctx->ev[r][i]));
    ctx->timing = value != 0;
    ctx->ev_count = 0;
  } else if (!strcmp(name, "graph")) {
    ctx->use_graph = value != 0;
    if (!ctx->use_graph) drop_graphs(ctx);
  } else if (!strcmp(name, "persist.grid")) ctx->persist_grid = value;
  else if (!strcmp(name, "persist.hmax")) ctx->persist_hmax = value;
  else if (!strcmp(name, "mldsa.internal")) {
    if (value != 0 && value != 1) return fail(ctx, DIL_EINVAL, "mldsa.internal must be 0 or 1");
    ctx->mldsa_internal = (int)value;
  } else if (!strcmp(name, "persist.tail")) {
    if (value < -1 || value > 64) return fail(ctx, DIL_EINVAL, "persist.tail must be -1..64");
    ctx->persist_tail = (int)value;
  }
  else if (!strcmp(name, "persist.waves")) {
    if (value != 1 && value != 2 && value != 4) return fail(ctx, DIL_EINVAL, "persist.waves must be 1, 2 or 4");
    ctx->persist_waves = (int)value;
  } else if (!strcmp(name, "ntt.variant")) {
    if (value < 0 || value > 3) return fail(ctx, DIL_EINVAL, "ntt.variant must be 0..3");
    ctx->ntt_variant = (int)value;
  } else if (!strcmp(name, "t0.variant")) {
    if (value < 0 || value > 3) return fail(ctx, DIL_EINVAL, "t0.variant must be 0..3");
    ctx->t0_variant = (int)value;
  } else if (!strcmp(name, "persist.pad")) {
    if (value != 0 && value != 1) return fail(ctx, DIL_EINVAL, "persist.pad must be 0 or 1");
    ctx->persist_pad = (int)value;
  }
  else return fail(ctx, DIL_EINVAL, "unknown parameter");
  return DIL_OK;
}

int dil_sizes(int level, size_t *pk, size_t *sk, size_t *sig) {
  return by_level(level, [&](auto lv) {
    constexpr int LV = decltype(lv)::value;
    if (pk) *pk = P<LV>::PK;
    if (sk) *sk = P<LV>::SK;
    if (sig) *sig = P<LV>::SIG;
    return DIL_OK;
  });
}

int dil_keygen_batch(dil_ctx *ctx, int level, const uint8_t *seeds, uint8_t *pk, uint8_t *sk, uint32_t count,
                     void *stream) {
  if (!ctx || !valid_level(level)) return fail(ctx, DIL_EINVAL, "bad context or level");
  if (count == 0) return DIL_OK;
  if (!seeds || !pk || !sk) return fail(ctx, DIL_EINVAL, "null buffer");
  hipSetDevice(ctx->device);
  return by_level(level, [&](auto lv) {
    return keygen_impl<decltype(lv)::value>(ctx, seeds, pk, sk, count, (hipStream_t)stream);
  });
}

int dil_sign_batch(dil_ctx *ctx, int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                   const uint64_t *msg_off, uint8_t *sig, uint32_t count, void *stream) {
  return dil_sign_batch_rnd(ctx, level, sk, key_idx, msg, msg_off, nullptr, sig, count, stream);
}

int dil_sign_batch_rnd(dil_ctx *ctx, int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                       const uint64_t *msg_off, const uint8_t *rnd, uint8_t *sig, uint32_t count, void *stream) {
  if (!ctx || !valid_level(level)) return fail(ctx, DIL_EINVAL, "bad context or level");
  if (count == 0) return DIL_OK;
  if (!sk || !msg || !msg_off || !sig) return fail(ctx, DIL_EINVAL, "null buffer");
  if ((uintptr_t)rnd & 3) return fail(ctx, DIL_EINVAL, "rnd must be 4-byte aligned");
  if (check_form(ctx, level)) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  ctx->stats_pending = 0;
  return by_level(level, [&](auto lv) {
    if (ctx->mode == DIL_MODE_PERSISTENT)
      return sign_persistent<decltype(lv)::value>(ctx, sk, key_idx, msg, msg_off, sig, count, (hipStream_t)stream,
                                                  nullptr, rnd);
    return sign_staged<decltype(lv)::value>(ctx, sk, key_idx, msg, msg_off, sig, count, (hipStream_t)stream, nullptr,
                                            rnd);
  });
}

int dil_verify_batch(dil_ctx *ctx, int level, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                     const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count, void *stream) {
  if (!ctx || !valid_level(level)) return fail(ctx, DIL_EINVAL, "bad context or level");
  if (count == 0) return DIL_OK;
  if (!pk || !msg || !msg_off || !sig || !verdict) return fail(ctx, DIL_EINVAL, "null buffer");
  if (check_form(ctx, level)) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  return by_level(level, [&](auto lv) {
    return verify_impl<decltype(lv)::value>(ctx, pk, key_idx, msg, msg_off, sig, verdict, count,
                                            (hipStream_t)stream);
  });
}

int dil_keyset_create(dil_ctx *ctx, int level, const uint8_t *pk, const uint8_t *sk, uint32_t n_keys,
                      dil_keyset **out, void *stream) {
  if (!ctx || !out || !valid_level(level) || n_keys == 0 || (!pk && !sk))
    return fail(ctx, DIL_EINVAL, "bad key table arguments");
  *out = nullptr;
  hipSetDevice(ctx->device);
  dil_keyset *ks = new dil_keyset();
  ks->level = level;
  ks->nkeys = n_keys;
  ks->device = ctx->device;
  int rc = by_level(level, [&](auto lv) {
    return keyset_build<decltype(lv)::value>(ctx, ks, pk, sk, (hipStream_t)stream);
  });
  if (rc) {
    if (ks->mem) hipFree(ks->mem);
    delete ks;
    return rc;
  }
  *out = ks;
  return DIL_OK;
}

int dil_keyset_destroy(dil_keyset *ks) {
  if (!ks) return DIL_EINVAL;
  hipSetDevice(ks->device);
  hipDeviceSynchronize();
  if (ks->mem) hipFree(ks->mem);
  delete ks;
  return DIL_OK;
}

int dil_keyset_info(const dil_keyset *ks, int *level, uint32_t *n_keys, size_t *device_bytes) {
  if (!ks) return DIL_EINVAL;
  if (level) *level = ks->level;
  if (n_keys) *n_keys = ks->nkeys;
  if (device_bytes) *device_bytes = ks->bytes;
  return DIL_OK;
}

int dil_sign_keyset(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                    const uint64_t *msg_off, uint8_t *sig, uint32_t count, void *stream) {
  if (!ctx || !ks) return fail(ctx, DIL_EINVAL, "bad context or key table");
  if (!ks->sk) return fail(ctx, DIL_EINVAL, "key table holds no secret keys");
  if (count == 0) return DIL_OK;
  if (!msg || !msg_off || !sig) return fail(ctx, DIL_EINVAL, "null buffer");
  if (!key_idx && count > ks->nkeys) return fail(ctx, DIL_EINVAL, "more tasks than keys without key_idx");
  if (check_form(ctx, ks->level)) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  ctx->stats_pending = 0;
  return by_level(ks->level, [&](auto lv) {
    constexpr int LV = decltype(lv)::value;
    if (ctx->mode == DIL_MODE_PERSISTENT)
      return sign_persistent<LV>(ctx, ks->sk, key_idx, msg, msg_off, sig, count, (hipStream_t)stream, ks);
    return sign_staged<LV>(ctx, ks->sk, key_idx, msg, msg_off, sig, count, (hipStream_t)stream, ks);
  });
}

}  // extern "C"

namespace {
// dil_verify_keyset's kernels over the scratch array: the same launches on
// `st` as a key-table Verify (no side streams, no graph), with the workspace
// laid out in the scratch array instead of the context's pool.
template <int LV>
int verify_keyset_noalloc_impl(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                               const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                               hipStream_t st) {
  const size_t need = ws_layout<LV>(nullptr, count, WS_VERIFY, true, 0, 1, nullptr, nullptr, nullptr);
  if (need > NOALLOC_SCRATCH_BYTES) {
    char t[160];
    snprintf(t, sizeof t, "count %u needs %zu bytes of scratch, above the %zu-byte maximum", count, need,
             NOALLOC_SCRATCH_BYTES);
    return fail(ctx, DIL_EINVAL, t);
  }
  Ws ws;
  uint32_t *kid = nullptr;
  ws_layout<LV>(ctx->scratch, count, WS_VERIFY, true, 0, 1, &ws, nullptr, &kid);
  ws.kmap = nullptr;
  ws.t1h = nullptr;
  ws.tr = nullptr;
  const uint32_t *kidx = use_keyset(ws, ks, key_idx, kid);
  zero_words_k<<<1, 64, 0, st>>>(ws.counters, 16, nullptr, 0);
  check_keys(ctx, ks, key_idx, kid, count, st);
  launch_vf_hash<LV>(ctx, st, ks->pk, kidx, msg, msg_off, ws, count, ctx->dev_stats + ERR_WORD_MSG);
  vf_prep_k<LV><<<blocks_for(count, 64), 64, 0, st>>>(sig, ws, count);
  vf_main_k<LV><<<count, 64, 0, st>>>(ks->pk, kidx, sig, ws, count);
  vf_final_k<LV><<<blocks_for(2 * (uint64_t)count, 256), 256, 0, st>>>(sig, ws, verdict, count);
  LAUNCHCHK(ctx);
  return DIL_OK;
}
}  // namespace

extern "C" {

int dil_verify_keyset_noalloc(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                              const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                              void *stream) {
  if (!ctx || !ks) return fail(ctx, DIL_EINVAL, "bad context or key table");
  if (!ks->pk) return fail(ctx, DIL_EINVAL, "key table holds no public keys");
  if (ks->device != ctx->device) return fail(ctx, DIL_EINVAL, "key table and context on different devices");
  if (count == 0) return DIL_OK;
  if (!msg || !msg_off || !sig || !verdict) return fail(ctx, DIL_EINVAL, "null buffer");
  if (!key_idx && count > ks->nkeys) return fail(ctx, DIL_EINVAL, "more tasks than keys without key_idx");
  if (check_form(ctx, ks->level)) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  return by_level(ks->level, [&](auto lv) {
    return verify_keyset_noalloc_impl<decltype(lv)::value>(ctx, ks, key_idx, msg, msg_off, sig, verdict, count,
                                                           (hipStream_t)stream);
  });
}

int dil_verify_keyset(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                      const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count, void *stream) {
  if (!ctx || !ks) return fail(ctx, DIL_EINVAL, "bad context or key table");
  if (!ks->pk) return fail(ctx, DIL_EINVAL, "key table holds no public keys");
  if (count == 0) return DIL_OK;
  if (!msg || !msg_off || !sig || !verdict) return fail(ctx, DIL_EINVAL, "null buffer");
  if (!key_idx && count > ks->nkeys) return fail(ctx, DIL_EINVAL, "more tasks than keys without key_idx");
  if (check_form(ctx, ks->level)) return DIL_EINVAL;
  hipSetDevice(ctx->device);
  return by_level(ks->level, [&](auto lv) {
    return verify_impl<decltype(lv)::value>(ctx, ks->pk, key_idx, msg, msg_off, sig, verdict, count,
                                            (hipStream_t)stream, ks);
  });
}

}  // extern "C"

namespace {
// workspace bytes of one call (op DIL_OP_*, resident key table or not) of
// `count` tasks in the context's current Sign form and schedule knobs; with
// `upto` the layout covers every call of at most `count` tasks
template <int LV>
int call_bytes(dil_ctx *ctx, int op, bool keyset, uint32_t count, bool upto, size_t *bytes) {
  if (op == DIL_OP_KEYGEN) {
    *bytes = ws_layout<LV>(nullptr, count, WS_KEYGEN, false, 0, 1, nullptr, nullptr, nullptr);
  } else if (op == DIL_OP_VERIFY) {
    *bytes = ws_layout<LV>(nullptr, count, WS_VERIFY, keyset, 0, 1, nullptr, nullptr, nullptr);
  } else if (op == DIL_OP_SIGN && ctx->mode == DIL_MODE_STAGED) {
    *bytes = ws_layout<LV>(nullptr, count, WS_SIGN_STAGED, keyset, 0, 1, nullptr, nullptr, nullptr);
  } else if (op == DIL_OP_SIGN) {
    uint64_t grid = 1, hmax = 1;
    int rc = persist_schedule<LV>(ctx, count, &grid, &hmax);
    if (rc) return rc;
    if (upto && ctx->persist_grid <= 0) {  // smaller calls launch at most min(count, resident) workgroups
      int occ = 1;
      rc = persist_occupancy<LV>(ctx, &occ);
      if (rc) return rc;
      grid = std::max<uint64_t>(grid, std::min<uint64_t>(std::max<uint32_t>(count, 1), (uint64_t)occ * ctx->cu_count));
    }
    *bytes = ws_layout<LV>(nullptr, count, WS_SIGN_PERSIST, keyset, grid, ctx->persist_waves, nullptr, nullptr,
                           nullptr);
  } else {
    return fail(ctx, DIL_EINVAL, "op must be DIL_OP_KEYGEN, DIL_OP_SIGN or DIL_OP_VERIFY");
  }
  return DIL_OK;
}
}  // namespace

extern "C" {

int dil_workspace_bytes(dil_ctx *ctx, int level, int op, int keyset, uint32_t count, size_t *bytes) {
  if (!ctx || !valid_level(level) || !bytes) return fail(ctx, DIL_EINVAL, "bad context, level or output");
  hipSetDevice(ctx->device);
  return by_level(level, [&](auto lv) { return call_bytes<decltype(lv)::value>(ctx, op, keyset != 0, count, false, bytes); });
}

int dil_ctx_reserve_call(dil_ctx *ctx, int level, int op, int keyset, uint32_t count) {
  if (!ctx || !valid_level(level)) return fail(ctx, DIL_EINVAL, "bad context or level");
  hipSetDevice(ctx->device);
  size_t need = 0;
  int rc = by_level(level, [&](auto lv) { return call_bytes<decltype(lv)::value>(ctx, op, keyset != 0, count, true, &need); });
  if (rc) return rc;
  rc = ws_reserve_bytes(ctx, need, nullptr);
  if (rc) return rc;
  HIPCHK(ctx, hipStreamSynchronize(nullptr));
  return DIL_OK;
}

int dil_ctx_reserve(dil_ctx *ctx, int level, uint32_t count) {
  if (!ctx || !valid_level(level)) return fail(ctx, DIL_EINVAL, "bad context or level");
  hipSetDevice(ctx->device);
  size_t need = 0;
  const int saved = ctx->mode;
  int rc = DIL_OK;
  for (int op = DIL_OP_KEYGEN; op <= DIL_OP_VERIFY && !rc; op++)
    for (int ks = 0; ks < 2 && !rc; ks++)
      for (int m = DIL_MODE_STAGED; m <= DIL_MODE_PERSISTENT && !rc; m++) {
        ctx->mode = m;
        size_t b = 0;
        rc = by_level(level, [&](auto lv) { return call_bytes<decltype(lv)::value>(ctx, op, ks != 0, count, true, &b); });
        need = std::max(need, b);
      }
  ctx->mode = saved;
  if (rc) return rc;
  rc = ws_reserve_bytes(ctx, need, nullptr);
  if (rc) return rc;
  HIPCHK(ctx, hipStreamSynchronize(nullptr));
  return DIL_OK;
}

int dil_persist_capacity(dil_ctx *ctx, int level, int *resident_groups, int *slots_per_batch) {
  if (!ctx || !valid_level(level)) return fail(ctx, DIL_EINVAL, "bad context or level");
  hipSetDevice(ctx->device);
  return by_level(level, [&](auto lv) {
    constexpr int LV = decltype(lv)::value;
    int occ = 1;
    int rc = persist_occupancy<LV>(ctx, &occ);
    if (rc) return rc;
    if (resident_groups) *resident_groups = occ * ctx->cu_count;
    if (slots_per_batch) *slots_per_batch = persist_slots<LV>(ctx->persist_waves);
    return DIL_OK;
  });
}

int dil_sign_timing(dil_ctx *ctx, float *setup_ms, float *loop_ms, int max_calls, int *n_calls) {
  if (!ctx) return DIL_EINVAL;
  int n = std::min(ctx->ev_count, dil_ctx::RING);
  if (max_calls < n) n = max_calls;
  if (n_calls) *n_calls = n;
  for (int k = 0; k < n; k++) {
    hipEvent_t *e = ctx->ev[(ctx->ev_count - n + k) % dil_ctx::RING];
    HIPCHK(ctx, hipEventSynchronize(e[2]));
    float a = 0, b = 0;
    HIPCHK(ctx, hipEventElapsedTime(&a, e[0], e[1]));
    HIPCHK(ctx, hipEventElapsedTime(&b, e[1], e[2]));
    if (setup_ms) setup_ms[k] = a;
    if (loop_ms) loop_ms[k] = b;
  }
  return DIL_OK;
}

#ifdef DIL_PHASE_TIMERS
// Development aid (phase-timer builds only): raw statistics words (64) of the context.
extern "C" int dil_debug_stats(dil_ctx *ctx, uint32_t *out64) {
  if (!ctx || !out64) return DIL_EINVAL;
  HIPCHK(ctx, hipDeviceSynchronize());
  HIPCHK(ctx, hipMemcpy(out64, ctx->dev_stats, 256, hipMemcpyDeviceToHost));
  return DIL_OK;
}
#endif

int dil_sign_stats(dil_ctx *ctx, uint64_t *evaluated, uint64_t *sequential) {
  if (!ctx) return DIL_EINVAL;
  if (ctx->stats_pending) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->last_stream));
    HIPCHK(ctx, hipMemcpy(ctx->host_counters, ctx->dev_stats, 32, hipMemcpyDeviceToHost));
    ctx->stat_evaluated = (uint64_t)ctx->host_counters[2] | ((uint64_t)ctx->host_counters[3] << 32);
    ctx->stat_sequential = (uint64_t)ctx->host_counters[6] | ((uint64_t)ctx->host_counters[7] << 32);
    ctx->stats_pending = 0;
    if (ctx->host_counters[5]) return fail(ctx, DIL_EHIP, "a task exceeded the iteration limit");
  }
  if (evaluated) *evaluated = ctx->stat_evaluated;
  if (sequential) *sequential = ctx->stat_sequential;
  return DIL_OK;
}

int dil_ntt_mul_batch(dil_ctx *ctx, const int32_t *a, const int32_t *b, int32_t *c, uint64_t count, void *stream) {
  if (!ctx) return DIL_EINVAL;
  if (count == 0) return DIL_OK;
  if (!a || !b || !c) return fail(ctx, DIL_EINVAL, "null buffer");
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return fail(ctx, DIL_EINVAL, "buffers must be 16-byte aligned");
  hipSetDevice(ctx->device);
  if (!ctx->cu_count) {
    hipDeviceProp_t prop;
    HIPCHK(ctx, hipGetDeviceProperties(&prop, ctx->device));
    ctx->cu_count = prop.multiProcessorCount;
  }
  // 16 polynomials per 256-lane workgroup, grid-strided over at most 16 workgroups per CU
  const uint64_t need = (count + 15) / 16;
  const unsigned grid = (unsigned)std::min<uint64_t>(need, (uint64_t)ctx->cu_count * 16);
  const hipStream_t st = (hipStream_t)stream;
  switch (ctx->ntt_variant) {
    case 0: ntt_mul_k<true><<<grid, 256, 0, st>>>(a, b, c, count); break;
    case 1: ntt_mul_k<false><<<grid, 256, 0, st>>>(a, b, c, count); break;
    case 2: ntt_mul_perlevel_k<<<grid, 256, 0, st>>>(a, b, c, count); break;
    default: {
      ntt_fwd_k<<<grid, 256, 0, st>>>(a, c, count);
      const uint64_t words4 = count * (N / 4);
      const unsigned pgrid = (unsigned)std::min<uint64_t>((words4 + 255) / 256, (uint64_t)ctx->cu_count * 16);
      ntt_pointwise_k<<<pgrid, 256, 0, st>>>(c, b, words4);
      ntt_inv_k<<<grid, 256, 0, st>>>(c, count);
    }
  }
  LAUNCHCHK(ctx);
  return DIL_OK;
}

int dil_alu_probe(dil_ctx *ctx, int kind, uint32_t iters, uint32_t groups, uint32_t *out, void *stream,
                  uint64_t *instructions) {
  if (!ctx || !out || groups == 0) return fail(ctx, DIL_EINVAL, "bad probe arguments");
  hipSetDevice(ctx->device);
  const hipStream_t st = (hipStream_t)stream;
  switch (kind) {
    case 0: alu_probe_k<0><<<groups, PROBE_WG, 0, st>>>(out, iters); break;
    case 1: alu_probe_k<1><<<groups, PROBE_WG, 0, st>>>(out, iters); break;
    case 2: alu_probe_k<2><<<groups, PROBE_WG, 0, st>>>(out, iters); break;
    case 3: alu_probe_k<3><<<groups, PROBE_WG, 0, st>>>(out, iters); break;
    case 4: alu_probe_k<4><<<groups, PROBE_WG, 0, st>>>(out, iters); break;
    case 5: alu_probe_k<5><<<groups, PROBE_WG, 0, st>>>(out, iters); break;
    default: return fail(ctx, DIL_EINVAL, "probe kind must be 0..5");
  }
  LAUNCHCHK(ctx);
  if (instructions) *instructions = (uint64_t)groups * PROBE_WG * iters * PROBE_INSTR_PER_ITER;
  return DIL_OK;
}

int dil_t0_ntt_batch(dil_ctx *ctx, int level, const uint8_t *sk, int32_t *t0_hat, uint32_t count, void *stream) {
  if (!ctx) return DIL_EINVAL;
  if (level != 2 && level != 3 && level != 5) return fail(ctx, DIL_EINVAL, "level must be 2, 3 or 5");
  if (count == 0) return DIL_OK;
  if (!sk || !t0_hat) return fail(ctx, DIL_EINVAL, "null buffer");
  if (((uintptr_t)sk & 7) || ((uintptr_t)t0_hat & 15))
    return fail(ctx, DIL_EINVAL, "sk must be 8-byte and t0_hat 16-byte aligned");
  hipSetDevice(ctx->device);
  const hipStream_t st = (hipStream_t)stream;
  const int variant = ctx->t0_variant;
  return by_round3_level(level, [&](auto lv) {
    constexpr int LV = decltype(lv)::value;
    switch (variant) {
      case 0: t0_ntt_reg_k<LV, true><<<count, 64, 0, st>>>(sk, t0_hat, count); break;
      case 1: t0_ntt_reg_k<LV, false><<<count, 64, 0, st>>>(sk, t0_hat, count); break;
      case 2: t0_ntt_gmem_k<LV, true><<<count, 64, 0, st>>>(sk, t0_hat, count); break;
      default:
        t0_unpack_k<LV><<<blocks_for((uint64_t)count * Lv<LV>::K * 32, 256), 256, 0, st>>>(sk, t0_hat, count);
        t0_ntt_gmem_k<LV, false><<<count, 64, 0, st>>>(sk, t0_hat, count);
    }
    LAUNCHCHK(ctx);
    return DIL_OK;
  });
}

int dil_expand_a_batch(dil_ctx *ctx, const uint8_t *seeds34, int32_t *out, uint64_t count, void *stream) {
  if (!ctx) return DIL_EINVAL;
  if (count == 0) return DIL_OK;
  if (!seeds34 || !out) return fail(ctx, DIL_EINVAL, "null buffer");
  if (count > (uint64_t)UINT32_MAX) return fail(ctx, DIL_EINVAL, "count above 2^32 - 1");
  hipSetDevice(ctx->device);
  expand_a_seed_k<<<blocks_for(count, EA_WG), EA_WG, 0, (hipStream_t)stream>>>(seeds34, out, count);
  LAUNCHCHK(ctx);
  return DIL_OK;
}

}  // extern "C"
