// Continuous-batching serving engine (host C++) over resident key tables.
//
// Requests -- Sign or Verify of one message against one key row of a level's
// dil_keyset -- become visible to the dispatcher at their arrival time.  The
// dispatcher keeps up to n_streams batches in flight, each on its own HIP
// stream with its own libdil contexts (workspaces) and pinned staging buffers.
// Device memory: at creation every lane reserves, for each (level, op) group,
// the workspace of a key-table call of C requests (dil_workspace_bytes), C the
// largest count for which all lanes' workspaces and device staging buffers fit
// the memory budget; no call allocates afterwards.  Whenever a stream is free
// the dispatcher admits the arrived requests in order while each (level, op)
// group of the batch holds at most C of them (and the messages fit the
// staging buffer); the next request waits for the next batch.  The batch is
// split by (level, op) into dil_sign_keyset / dil_verify_keyset calls, and the
// host->device copies, the kernels and the device->host copies are enqueued,
// followed by an event.
// The (level, op) groups of a batch are independent: each runs on a stream and
// context of its own, forked after the batch's copies in and joined before its
// copies out, so a batch takes about as long as its slowest group.  This
// needs hardware queues for the lanes' and groups' streams: with HIP's
// default of 4 per process they serialise, so serving processes should raise
// GPU_MAX_HW_QUEUES (the benchmark uses 16).
// Completed batches are harvested by polling the events; a request's
// completion time is the poll that observed its batch's event.
//
// Two ways in: dil_server_run replays a whole trace of timed arrivals on the
// calling thread, and the interactive mode (dil_server_start ... stop) runs the
// same dispatcher on a thread of its own, fed by dil_server_submit from any
// host thread; the caller collects each result once with dil_server_poll or
// dil_server_wait.  Both share the batch formation, staging and harvesting
// below; one server runs one of them at a time.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/dil.h"

namespace {

// the levels a server can hold tables for: round 3, then ML-DSA-44 / 65 / 87
constexpr int NLV = 6;
const int kLevels[NLV] = {2, 3, 5, 44, 65, 87};
int lv_index(int level) {
  for (int i = 0; i < NLV; i++)
    if (kLevels[i] == level) return i;
  return -1;
}

struct Group {
  int li, op;                 // level index, 0 sign / 1 verify
  std::vector<uint32_t> req;  // requests of the batch (index within the batch)
  size_t m_pos = 0, m_len = 0, t_pos = 0, o_pos = 0, s_pos = 0;
};

// A request of the interactive mode, with its own copies of the bytes.
struct SvcReq {
  uint64_t ticket = 0;
  int li = 0, op = 0;
  uint32_t key = 0;
  std::vector<uint8_t> msg, sig;
};

struct SvcRes {
  int32_t verdict = -1;      // Verify: 1 / 0; Sign: -1
  std::vector<uint8_t> sig;  // Sign: the signature
};

constexpr int NGROUP = 2 * NLV;  // (level, op) groups, index 2 * level index + op

struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr, fork = nullptr;
  hipStream_t gst[NGROUP] = {};
  dil_ctx *gctx[NGROUP] = {};
  hipEvent_t gev[NGROUP] = {};
  uint8_t *h_msg = nullptr, *h_sig = nullptr, *d_msg = nullptr, *d_sig = nullptr;
  uint64_t *h_off = nullptr, *d_off = nullptr;
  uint32_t *h_key = nullptr, *d_key = nullptr;
  int32_t *h_ver = nullptr, *d_ver = nullptr;
  bool busy = false;
  std::vector<Group> groups;
  uint32_t base = 0;             // dil_server_run: trace index of the batch's first request
  std::vector<SvcReq> inflight;  // interactive mode: the batch's requests
};

}  // namespace

struct dil_server {
  int device = 0;
  dil_keyset *ks[NLV] = {};
  size_t sig_bytes[NLV] = {};
  uint32_t max_batch = 0;
  uint32_t group_cap = 0;     // requests of one (level, op) group per batch (memory budget)
  size_t max_msg = 0, budget = 0, reserved = 0;
  std::vector<Lane> lanes;
  char err[256] = {0};
  // statistics of the last run (interactive mode: since dil_server_start)
  uint64_t batches = 0, overlapped = 0;
  double host_s = 0;
  // interactive mode; mu guards everything below and err while it is on
  std::mutex mu;
  std::condition_variable cv_done;  // results (or a dispatcher error) for waiters
  std::condition_variable cv_in;    // new requests (or stop) for the dispatcher
  std::thread svc;
  bool svc_on = false, svc_stop = false;
  int svc_rc = DIL_OK;              // the dispatcher's first error, returned by every later call
  uint64_t next_ticket = 1;
  std::deque<SvcReq> pending;
  std::unordered_set<uint64_t> outstanding;          // submitted, result not yet handed out
  std::unordered_map<uint64_t, SvcRes> results;
};

namespace {

int sfail(dil_server *s, int code, const char *what) {
  if (s) snprintf(s->err, sizeof s->err, "%s", what);
  return code;
}

// Device bytes one lane holds with every group context reserved for `cap`
// requests (workspaces as the library lays them out, plus the staging buffers).
int lane_bytes(dil_server *s, const Lane &ln, uint32_t cap, size_t staging, size_t *out) {
  size_t total = staging;
  for (int gi = 0; gi < NGROUP; gi++) {
    if (!ln.gctx[gi]) continue;
    size_t b = 0;
    int rc = dil_workspace_bytes(ln.gctx[gi], kLevels[gi / 2], gi % 2 ? DIL_OP_VERIFY : DIL_OP_SIGN, 1, cap, &b);
    if (rc) return rc;
    total += b;
  }
  *out = total;
  return DIL_OK;
}

// One request as the batch stager reads it.
struct ReqRef {
  int li, op;
  uint32_t key;
  const uint8_t *msg;
  uint64_t len;
  const uint8_t *sig;  // Verify: sig_bytes[li] bytes
};

// How many of the next `avail` requests (in order) one batch admits: at most
// max_batch, at most group_cap per (level, op) group (its workspace
// reservation), and messages within the staging buffer; the first request
// that does not fit waits for the next batch.  peek(i, &group, &len).
template <class Peek>
uint32_t admit_count(const dil_server *s, uint32_t avail, Peek peek) {
  uint32_t per_group[NGROUP] = {};
  size_t mbytes = 0;
  uint32_t n = 0;
  while (n < avail && n < s->max_batch) {
    int gi = 0;
    uint64_t ml = 0;
    peek(n, &gi, &ml);
    if (per_group[gi] == s->group_cap || mbytes + ml > s->max_msg) break;
    per_group[gi]++;
    mbytes += ml;
    n++;
  }
  return n;
}

// One request's byte copies into a lane's pinned staging buffers.
struct CopyDesc {
  const uint8_t *msg, *sig;
  uint64_t len, sig_len;
  uint8_t *msg_dst, *sig_dst;
};

// Run fn(lo, hi) over [0, n) in contiguous ranges: on the calling thread
// alone for small jobs, else split over a few short-lived threads (the
// batch's host copies are several MB at full batches and bound the
// dispatcher's rate on one thread; a thread costs tens of microseconds).
template <class Fn>
void parallel_ranges(size_t n, size_t bytes, Fn fn) {
  constexpr size_t kMinBytesPerThread = 512 * 1024;
  const size_t hw = std::max<size_t>(1, std::thread::hardware_concurrency());
  size_t t = std::min<size_t>({4, hw, bytes / kMinBytesPerThread, n});
  if (t <= 1) {
    fn((size_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(t - 1);
  const size_t per = (n + t - 1) / t;
  try {
    for (size_t i = 1; i < t; i++) {
      const size_t lo = std::min(n, i * per), hi = std::min(n, lo + per);
      th.emplace_back([=]() { fn(lo, hi); });
    }
  } catch (...) {  // no more threads: the remaining ranges on this one
    for (size_t i = 1 + th.size(); i < t; i++) {
      const size_t lo = std::min(n, i * per), hi = std::min(n, lo + per);
      fn(lo, hi);
    }
  }
  fn((size_t)0, std::min(n, per));
  for (auto &x : th) x.join();
}

// Stage the nreq requests of one batch (get(r), r < nreq) into the lane's
// pinned buffers, grouped by (level, op) in request order, and enqueue the
// copies in, one key-table call per group on the group's own stream (forked
// after the copies in, joined before the copies out), the copies out and the
// lane's event.  Marks the lane busy; *overlap tells whether another lane's
// batch was still in flight.
template <class Get>
int launch_batch(dil_server *s, Lane &ln, uint32_t nreq, Get get, bool *overlap) {
  // one pass buckets the requests by (level, op), each bucket in request order
  std::vector<uint32_t> bucket[NGROUP];
  for (uint32_t r = 0; r < nreq; r++) {
    const ReqRef q = get(r);
    bucket[2 * q.li + q.op].push_back(r);
  }
  ln.groups.clear();
  for (int gi = 0; gi < NGROUP; gi++) {
    if (bucket[gi].empty()) continue;
    Group g;
    g.li = gi / 2;
    g.op = gi % 2;
    g.req = std::move(bucket[gi]);
    ln.groups.push_back(std::move(g));
  }
  // offsets, keys and the copies' sources and destinations, then the byte
  // copies into the pinned staging buffers (disjoint, split over threads for
  // large batches)
  std::vector<CopyDesc> copies;
  copies.reserve(nreq);
  size_t m_pos = 0, t_pos = 0, o_pos = 0, s_pos = 0, bytes = 0;
  for (auto &g : ln.groups) {
    size_t ss = s->sig_bytes[g.li];
    g.m_pos = m_pos;
    g.t_pos = t_pos;
    g.o_pos = o_pos;
    g.s_pos = s_pos;
    uint64_t acc = 0;
    for (size_t j = 0; j < g.req.size(); j++) {
      const ReqRef q = get(g.req[j]);
      CopyDesc c;
      c.msg = q.msg;
      c.len = q.len;
      c.msg_dst = ln.h_msg + m_pos + acc;
      c.sig = g.op == 1 ? q.sig : nullptr;
      c.sig_len = g.op == 1 ? ss : 0;
      c.sig_dst = ln.h_sig + s_pos + j * ss;
      copies.push_back(c);
      bytes += c.len + c.sig_len;
      ln.h_off[o_pos + j] = acc;
      acc += q.len;
      ln.h_key[t_pos + j] = q.key;
    }
    ln.h_off[o_pos + g.req.size()] = acc;
    g.m_len = acc;
    m_pos += acc;
    t_pos += g.req.size();
    o_pos += g.req.size() + 1;
    s_pos += g.req.size() * ss;
  }
  parallel_ranges(copies.size(), bytes, [&](size_t lo, size_t hi) {
    for (size_t k = lo; k < hi; k++) {
      const CopyDesc &c = copies[k];
      if (c.len) memcpy(c.msg_dst, c.msg, c.len);
      if (c.sig_len) memcpy(c.sig_dst, c.sig, c.sig_len);
    }
  });
  bool ok = hipMemcpyAsync(ln.d_msg, ln.h_msg, std::max<size_t>(m_pos, 1), hipMemcpyHostToDevice, ln.st) ==
                hipSuccess &&
            hipMemcpyAsync(ln.d_off, ln.h_off, o_pos * 8, hipMemcpyHostToDevice, ln.st) == hipSuccess &&
            hipMemcpyAsync(ln.d_key, ln.h_key, t_pos * 4, hipMemcpyHostToDevice, ln.st) == hipSuccess &&
            (s_pos == 0 || hipMemcpyAsync(ln.d_sig, ln.h_sig, s_pos, hipMemcpyHostToDevice, ln.st) == hipSuccess);
  if (!ok) return sfail(s, DIL_EHIP, "host-to-device copy");
  if (hipEventRecord(ln.fork, ln.st) != hipSuccess) return sfail(s, DIL_EHIP, "fork");
  for (auto &g : ln.groups) {
    uint32_t cnt = (uint32_t)g.req.size();
    const int gi = 2 * g.li + g.op;
    hipStream_t gs = ln.gst[gi];
    dil_ctx *gc = ln.gctx[gi];
    if (hipStreamWaitEvent(gs, ln.fork, 0) != hipSuccess) return sfail(s, DIL_EHIP, "fork wait");
    int rc;
    if (g.op == 0)
      rc = dil_sign_keyset(gc, s->ks[g.li], ln.d_key + g.t_pos, ln.d_msg + g.m_pos, ln.d_off + g.o_pos,
                           ln.d_sig + g.s_pos, cnt, gs);
    else
      rc = dil_verify_keyset(gc, s->ks[g.li], ln.d_key + g.t_pos, ln.d_msg + g.m_pos, ln.d_off + g.o_pos,
                             ln.d_sig + g.s_pos, ln.d_ver + g.t_pos, cnt, gs);
    if (rc) {
      snprintf(s->err, sizeof s->err, "batch call: %s", dil_last_error(gc));
      return rc;
    }
    if (hipEventRecord(ln.gev[gi], gs) != hipSuccess || hipStreamWaitEvent(ln.st, ln.gev[gi], 0) != hipSuccess)
      return sfail(s, DIL_EHIP, "join");
  }
  ok = (s_pos == 0 || hipMemcpyAsync(ln.h_sig, ln.d_sig, s_pos, hipMemcpyDeviceToHost, ln.st) == hipSuccess) &&
       hipMemcpyAsync(ln.h_ver, ln.d_ver, t_pos * 4, hipMemcpyDeviceToHost, ln.st) == hipSuccess &&
       hipEventRecord(ln.ev, ln.st) == hipSuccess;
  if (!ok) return sfail(s, DIL_EHIP, "device-to-host copy");
  bool others_busy = false;  // launched while another batch is still in flight
  for (auto &other : s->lanes) others_busy |= &other != &ln && other.busy;
  *overlap = others_busy;
  ln.busy = true;
  return DIL_OK;
}

// Hand every request of the lane's finished batch to put(r, op, sig, sig
// bytes, verdict) (Sign: sig, verdict -1; Verify: no sig) and free the lane.
template <class Put>
void harvest_lane(dil_server *s, Lane &ln, Put put) {
  for (auto &g : ln.groups) {
    size_t ss = s->sig_bytes[g.li];
    for (size_t j = 0; j < g.req.size(); j++) {
      if (g.op == 0) put(g.req[j], 0, ln.h_sig + g.s_pos + j * ss, ss, -1);
      else put(g.req[j], 1, (const uint8_t *)nullptr, (size_t)0, ln.h_ver[g.t_pos + j]);
    }
  }
  ln.busy = false;
  ln.groups.clear();
}

// The interactive mode's dispatcher thread.
void svc_fail(dil_server *s, int code, const char *what) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->svc_rc == DIL_OK) {
    s->svc_rc = code;
    if (what) snprintf(s->err, sizeof s->err, "%s", what);
  }
  s->cv_done.notify_all();
}

void svc_loop_body(dil_server *s);

void svc_loop(dil_server *s) {
  try {
    svc_loop_body(s);
  } catch (...) {  // host allocation failure
    svc_fail(s, DIL_ENOMEM, "dispatcher: host allocation failed");
  }
}

void svc_loop_body(dil_server *s) {
  using clk = std::chrono::steady_clock;
  if (hipSetDevice(s->device) != hipSuccess) return svc_fail(s, DIL_EHIP, "hipSetDevice");
  auto last_progress = clk::now();
  for (;;) {
    bool progressed = false;
    // harvest
    for (auto &ln : s->lanes) {
      if (!ln.busy) continue;
      hipError_t q = hipEventQuery(ln.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return svc_fail(s, DIL_EHIP, "batch failed on the device");
      std::vector<std::pair<uint64_t, SvcRes>> out;
      out.reserve(ln.inflight.size());
      harvest_lane(s, ln, [&](uint32_t r, int op, const uint8_t *sig, size_t ss, int32_t v) {
        SvcRes res;
        res.verdict = v;
        if (op == 0) res.sig.assign(sig, sig + ss);
        out.emplace_back(ln.inflight[r].ticket, std::move(res));
      });
      ln.inflight.clear();
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &o : out) s->results.emplace(o.first, std::move(o.second));
      }
      s->cv_done.notify_all();
      progressed = true;
    }
    // admit
    Lane *free_lane = nullptr;
    bool busy = false;
    for (auto &ln : s->lanes) {
      busy |= ln.busy;
      if (!ln.busy && !free_lane) free_lane = &ln;
    }
    std::vector<SvcReq> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (free_lane && !s->pending.empty()) {
        const uint32_t n = admit_count(s, (uint32_t)std::min<size_t>(s->pending.size(), UINT32_MAX),
                                       [&](uint32_t i, int *gi, uint64_t *len) {
                                         *gi = 2 * s->pending[i].li + s->pending[i].op;
                                         *len = s->pending[i].msg.size();
                                       });
        batch.assign(std::make_move_iterator(s->pending.begin()), std::make_move_iterator(s->pending.begin() + n));
        s->pending.erase(s->pending.begin(), s->pending.begin() + n);
      } else if (!busy && !progressed) {
        if (s->svc_stop && s->pending.empty()) return;
        // idle: wait for a submission (or stop); bounded so that stop is seen
        s->cv_in.wait_for(lk, std::chrono::milliseconds(2));
        last_progress = clk::now();
        continue;
      }
    }
    if (!batch.empty()) {
      auto h0 = clk::now();
      free_lane->inflight = std::move(batch);
      const std::vector<SvcReq> &b = free_lane->inflight;
      bool overlap = false;
      int rc = launch_batch(s, *free_lane, (uint32_t)b.size(), [&](uint32_t r) {
        return ReqRef{b[r].li, b[r].op, b[r].key, b[r].msg.data(), (uint64_t)b[r].msg.size(), b[r].sig.data()};
      }, &overlap);
      if (rc) return svc_fail(s, rc, nullptr);
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->batches++;
        s->overlapped += overlap ? 1 : 0;
        s->host_s += std::chrono::duration<double>(clk::now() - h0).count();
      }
      progressed = true;
    }
    if (progressed) {
      last_progress = clk::now();
    } else {
      if (clk::now() - last_progress > std::chrono::seconds(60)) return svc_fail(s, DIL_EHIP, "no batch completed for 60 s");
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

}  // namespace

extern "C" {

int dil_server_create_tables(dil_server **out, int device, dil_keyset *const *tables, int n_tables, int n_streams,
                             uint32_t max_batch, size_t max_msg_bytes, size_t mem_budget, int mode) {
  if (!out || n_tables < 0 || (n_tables && !tables) || n_streams < 1 || max_batch < 1 || max_msg_bytes < 1)
    return DIL_EINVAL;
  *out = nullptr;
  dil_keyset *by_level[NLV] = {};
  for (int i = 0; i < n_tables; i++) {
    int level = 0;
    if (!tables[i] || dil_keyset_info(tables[i], &level, nullptr, nullptr) != DIL_OK) return DIL_EINVAL;
    const int li = lv_index(level);
    if (li < 0 || by_level[li]) return DIL_EINVAL;  // one table per level
    by_level[li] = tables[i];
  }
  const int ctx_mode = mode & 0xFF;
  const bool mldsa_internal = (mode & DIL_SERVER_MLDSA_INTERNAL) != 0;
  if ((mode & ~(0xFF | DIL_SERVER_MLDSA_INTERNAL)) || (ctx_mode != DIL_MODE_STAGED && ctx_mode != DIL_MODE_PERSISTENT))
    return DIL_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return DIL_EHIP;
  dil_server *s = new dil_server();
  s->device = device;
  for (int i = 0; i < NLV; i++) s->ks[i] = by_level[i];
  s->max_batch = max_batch;
  s->max_msg = max_msg_bytes;
  s->budget = mem_budget;
  size_t max_sig = 0;
  for (int i = 0; i < NLV; i++) {
    size_t a, b, c;
    dil_sizes(kLevels[i], &a, &b, &c);
    s->sig_bytes[i] = c;
    max_sig = std::max(max_sig, c);
  }
  s->lanes.resize(n_streams);
  for (auto &ln : s->lanes) {
    bool ok = hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ln.fork, hipEventDisableTiming) == hipSuccess;
    for (int gi = 0; ok && gi < NGROUP; gi++) {
      int li = gi / 2;
      if (!s->ks[li]) continue;
      ok = hipStreamCreateWithFlags(&ln.gst[gi], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&ln.gev[gi], hipEventDisableTiming) == hipSuccess &&
           dil_ctx_create(&ln.gctx[gi], device, 0) == DIL_OK && dil_ctx_set_mode(ln.gctx[gi], ctx_mode) == DIL_OK &&
           // a group call holds few tasks: four-wavefront workgroups give each
           // task 4 x 64 / l nonces per batch, so almost every task passes in
           // the first batch instead of needing a second or third
           (gi % 2 == 1 || dil_ctx_set_param(ln.gctx[gi], "persist.waves", 4) == DIL_OK) &&
           // ML-DSA groups on formatted messages M' when asked (round-3 calls have no such form)
           (!mldsa_internal || kLevels[li] < 44 || dil_ctx_set_param(ln.gctx[gi], "mldsa.internal", 1) == DIL_OK);
    }
    ok = ok && hipHostMalloc((void **)&ln.h_msg, max_msg_bytes, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void **)&ln.h_sig, max_batch * max_sig, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void **)&ln.h_off, (max_batch + 8) * 8, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void **)&ln.h_key, max_batch * 4, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void **)&ln.h_ver, max_batch * 4, hipHostMallocDefault) == hipSuccess &&
         hipMalloc((void **)&ln.d_msg, max_msg_bytes) == hipSuccess &&
         hipMalloc((void **)&ln.d_sig, max_batch * max_sig) == hipSuccess &&
         hipMalloc((void **)&ln.d_off, (max_batch + 8) * 8) == hipSuccess &&
         hipMalloc((void **)&ln.d_key, max_batch * 4) == hipSuccess &&
         hipMalloc((void **)&ln.d_ver, max_batch * 4) == hipSuccess;
    if (!ok) {
      dil_server_destroy(s);
      return DIL_ENOMEM;
    }
  }
  // the largest per-group request count whose reservations fit the budget
  const size_t staging = max_msg_bytes + max_batch * max_sig + 2 * (max_batch + 8) * 8 + 2 * max_batch * 4;
  auto fits = [&](uint32_t cap, bool *ok) {
    size_t per = 0;
    if (lane_bytes(s, s->lanes[0], cap, staging, &per)) return DIL_EHIP;
    *ok = per * s->lanes.size() <= mem_budget;
    return DIL_OK;
  };
  uint32_t lo = 0, hi = max_batch;  // lo fits (0 = nothing fits yet), hi + 1 does not
  for (uint32_t probe = 1; lo < hi; probe = lo + (hi - lo + 1) / 2) {
    bool ok = false;
    if (fits(probe, &ok)) {
      dil_server_destroy(s);
      return DIL_EHIP;
    }
    if (ok) lo = probe;
    else hi = probe - 1;
  }
  if (lo == 0) {
    dil_server_destroy(s);
    return DIL_ENOMEM;  // not even one request per group fits the budget
  }
  s->group_cap = lo;
  for (auto &ln : s->lanes)
    for (int gi = 0; gi < NGROUP; gi++)
      if (ln.gctx[gi] && dil_ctx_reserve_call(ln.gctx[gi], kLevels[gi / 2], gi % 2 ? DIL_OP_VERIFY : DIL_OP_SIGN, 1,
                                              lo) != DIL_OK) {
        dil_server_destroy(s);
        return DIL_ENOMEM;
      }
  size_t per = 0;
  lane_bytes(s, s->lanes[0], lo, staging, &per);
  s->reserved = per * s->lanes.size();
  *out = s;
  return DIL_OK;
}

int dil_server_create(dil_server **out, int device, dil_keyset *ks2, dil_keyset *ks3, dil_keyset *ks5,
                      int n_streams, uint32_t max_batch, size_t max_msg_bytes, size_t mem_budget, int mode) {
  dil_keyset *tables[3];
  int n = 0;
  for (dil_keyset *k : {ks2, ks3, ks5})
    if (k) tables[n++] = k;
  return dil_server_create_tables(out, device, tables, n, n_streams, max_batch, max_msg_bytes, mem_budget, mode);
}

int dil_server_destroy(dil_server *s) {
  if (!s) return DIL_EINVAL;
  bool on;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    on = s->svc_on;
  }
  if (on) dil_server_stop(s);
  hipSetDevice(s->device);
  hipDeviceSynchronize();
  for (auto &ln : s->lanes) {
    for (int gi = 0; gi < NGROUP; gi++) {
      if (ln.gctx[gi]) dil_ctx_destroy(ln.gctx[gi]);
      if (ln.gev[gi]) hipEventDestroy(ln.gev[gi]);
      if (ln.gst[gi]) hipStreamDestroy(ln.gst[gi]);
    }
    if (ln.fork) hipEventDestroy(ln.fork);
    if (ln.ev) hipEventDestroy(ln.ev);
    if (ln.st) hipStreamDestroy(ln.st);
    hipHostFree(ln.h_msg);
    hipHostFree(ln.h_sig);
    hipHostFree(ln.h_off);
    hipHostFree(ln.h_key);
    hipHostFree(ln.h_ver);
    hipFree(ln.d_msg);
    hipFree(ln.d_sig);
    hipFree(ln.d_off);
    hipFree(ln.d_key);
    hipFree(ln.d_ver);
  }
  delete s;
  return DIL_OK;
}

const char *dil_server_last_error(dil_server *s) { return s ? s->err : "null server"; }

int dil_server_stats(dil_server *s, uint64_t *batches, double *host_seconds, uint64_t *overlapped,
                     uint32_t *group_cap, size_t *reserved_bytes) {
  if (!s) return DIL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (batches) *batches = s->batches;
  if (host_seconds) *host_seconds = s->host_s;
  if (overlapped) *overlapped = s->overlapped;
  if (group_cap) *group_cap = s->group_cap;
  if (reserved_bytes) *reserved_bytes = s->reserved;
  return DIL_OK;
}

int dil_server_run(dil_server *s, uint32_t n, const uint8_t *op, const uint8_t *level, const uint32_t *key,
                   const uint8_t *msg, const uint64_t *msg_off, const uint8_t *sig_in, const uint64_t *sig_in_off,
                   const uint64_t *arrival_ns, uint8_t *sig_out, const uint64_t *sig_out_off, int32_t *verdict,
                   uint64_t *done_ns) {
  if (!s) return DIL_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->svc_on) return sfail(s, DIL_EINVAL, "the interactive mode is on (dil_server_stop first)");
  }
  if (n == 0) return DIL_OK;
  if (!op || !level || !key || !msg || !msg_off || !arrival_ns || !verdict || !done_ns) return sfail(s, DIL_EINVAL, "null array");
  hipSetDevice(s->device);
  uint32_t nkeys[NLV] = {};
  for (int li = 0; li < NLV; li++)
    if (s->ks[li]) dil_keyset_info(s->ks[li], nullptr, &nkeys[li], nullptr);
  for (uint32_t i = 0; i < n; i++) {
    int li = lv_index(level[i]);
    if (li < 0 || !s->ks[li] || op[i] > 1) return sfail(s, DIL_EINVAL, "request names an unknown level or op");
    // key rows are read on the device without bounds checks
    if (key[i] >= nkeys[li]) return sfail(s, DIL_EINVAL, "request names a key row outside its level's table");
    if (i && arrival_ns[i] < arrival_ns[i - 1]) return sfail(s, DIL_EINVAL, "arrivals must be sorted");
    if (msg_off[i + 1] < msg_off[i] || msg_off[i + 1] - msg_off[i] > s->max_msg)
      return sfail(s, DIL_EINVAL, "bad message offset or message larger than the staging buffer");
    if (op[i] == 0 && (!sig_out || !sig_out_off)) return sfail(s, DIL_EINVAL, "sign request without output");
    if (op[i] == 1 && (!sig_in || !sig_in_off)) return sfail(s, DIL_EINVAL, "verify request without signature");
  }
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now_ns = [&]() { return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - t0).count(); };
  s->batches = s->overlapped = 0;
  s->host_s = 0;
  uint32_t head = 0, done = 0;
  auto last_progress = clk::now();
  while (done < n) {
    bool progressed = false;
    if (clk::now() - last_progress > std::chrono::seconds(60)) return sfail(s, DIL_EHIP, "no batch completed for 60 s");
    // harvest
    for (auto &ln : s->lanes) {
      if (!ln.busy) continue;
      hipError_t q = hipEventQuery(ln.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return sfail(s, DIL_EHIP, "batch failed on the device");
      const uint64_t t = now_ns();
      std::vector<CopyDesc> outs;  // signatures out of the lane's staging buffer
      size_t bytes = 0;
      harvest_lane(s, ln, [&](uint32_t r, int o, const uint8_t *sig, size_t ss, int32_t v) {
        const uint32_t i = ln.base + r;
        done_ns[i] = t;
        if (o == 0) {
          outs.push_back(CopyDesc{sig, nullptr, ss, 0, sig_out + sig_out_off[i], nullptr});
          bytes += ss;
        }
        verdict[i] = v;
        done++;
      });
      // the lane is reused only after this loop, so its staging buffer still holds them
      parallel_ranges(outs.size(), bytes, [&](size_t lo, size_t hi) {
        for (size_t k = lo; k < hi; k++) memcpy(outs[k].msg_dst, outs[k].msg, outs[k].len);
      });
      progressed = true;
    }
    // admit the arrived requests into a free lane
    const uint64_t tnow = now_ns();
    const uint32_t arrived = (uint32_t)(std::upper_bound(arrival_ns, arrival_ns + n, tnow) - arrival_ns);
    Lane *free_lane = nullptr;
    for (auto &ln : s->lanes)
      if (!ln.busy) {
        free_lane = &ln;
        break;
      }
    if (free_lane && head < arrived) {
      auto h0 = clk::now();
      const uint32_t cnt = admit_count(s, arrived - head, [&](uint32_t k, int *gi, uint64_t *len) {
        const uint32_t r = head + k;
        *gi = 2 * lv_index(level[r]) + op[r];
        *len = msg_off[r + 1] - msg_off[r];
      });
      if (cnt) {
        free_lane->base = head;
        bool overlap = false;
        int rc = launch_batch(s, *free_lane, cnt, [&](uint32_t k) {
          const uint32_t r = head + k;
          return ReqRef{lv_index(level[r]), op[r], key[r], msg + msg_off[r], msg_off[r + 1] - msg_off[r],
                        op[r] == 1 ? sig_in + sig_in_off[r] : nullptr};
        }, &overlap);
        if (rc) return rc;
        s->batches++;
        s->overlapped += overlap ? 1 : 0;
        head += cnt;
        progressed = true;
        s->host_s += std::chrono::duration<double>(clk::now() - h0).count();
      }
    }
    if (progressed) last_progress = clk::now();
    if (!progressed) {
      bool any_busy = false;
      for (auto &ln : s->lanes) any_busy |= ln.busy;
      if (!any_busy) last_progress = clk::now();  // idle between arrivals is not a stall
      if (!any_busy && head < n) {
        uint64_t t = now_ns();
        if (arrival_ns[head] > t) std::this_thread::sleep_for(std::chrono::nanoseconds(std::min<uint64_t>(arrival_ns[head] - t, 200000)));
      } else {
        std::this_thread::yield();
      }
    }
  }
  return DIL_OK;
}

int dil_server_start(dil_server *s) {
  if (!s) return DIL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->svc_on) return sfail(s, DIL_EINVAL, "the interactive mode is already on");
  s->svc_stop = false;
  s->svc_rc = DIL_OK;
  s->pending.clear();
  s->outstanding.clear();
  s->results.clear();
  s->batches = s->overlapped = 0;
  s->host_s = 0;
  try {
    s->svc = std::thread(svc_loop, s);
  } catch (...) {
    return sfail(s, DIL_EHIP, "cannot start the dispatcher thread");
  }
  s->svc_on = true;
  return DIL_OK;
}

int dil_server_submit(dil_server *s, int op, int level, uint32_t key, const uint8_t *msg, uint64_t msg_len,
                      const uint8_t *sig, uint64_t *ticket) {
  if (!s || !ticket) return DIL_EINVAL;
  const int li = lv_index(level);
  if (li < 0 || !s->ks[li] || (op != 0 && op != 1) || (msg_len && !msg) || (op == 1 && !sig))
    return DIL_EINVAL;
  uint32_t nkeys = 0;
  dil_keyset_info(s->ks[li], nullptr, &nkeys, nullptr);
  if (key >= nkeys || msg_len > s->max_msg) return DIL_EINVAL;  // key rows are read without bounds checks
  try {
    SvcReq q;
    q.li = li;
    q.op = op;
    q.key = key;
    q.msg.assign(msg, msg + msg_len);
    if (op == 1) q.sig.assign(sig, sig + s->sig_bytes[li]);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->svc_rc) return s->svc_rc;
    if (!s->svc_on || s->svc_stop) return DIL_EINVAL;
    q.ticket = s->next_ticket;
    s->outstanding.insert(q.ticket);
    s->pending.push_back(std::move(q));
    *ticket = s->next_ticket++;
  } catch (...) {
    return DIL_ENOMEM;
  }
  s->cv_in.notify_one();
  return DIL_OK;
}

namespace {
// hand out a finished result (called with mu held)
void take_result(dil_server *s, uint64_t ticket, int32_t *verdict, uint8_t *sig_out) {
  auto it = s->results.find(ticket);
  if (verdict) *verdict = it->second.verdict;
  if (sig_out && !it->second.sig.empty()) memcpy(sig_out, it->second.sig.data(), it->second.sig.size());
  s->results.erase(it);
  s->outstanding.erase(ticket);
}
}  // namespace

int dil_server_poll(dil_server *s, uint64_t ticket, int *done, int32_t *verdict, uint8_t *sig_out) {
  if (!s || !done) return DIL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *done = 0;
  if (!s->outstanding.count(ticket)) return DIL_EINVAL;
  if (s->results.count(ticket)) {
    take_result(s, ticket, verdict, sig_out);
    *done = 1;
    return DIL_OK;
  }
  return s->svc_rc;
}

int dil_server_wait(dil_server *s, uint64_t ticket, int32_t timeout_ms, int32_t *verdict, uint8_t *sig_out) {
  if (!s) return DIL_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->outstanding.count(ticket)) return DIL_EINVAL;
  auto ready = [&]() { return s->results.count(ticket) || s->svc_rc != DIL_OK || !s->svc_on; };
  if (timeout_ms < 0) s->cv_done.wait(lk, ready);
  else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  if (s->results.count(ticket)) {
    take_result(s, ticket, verdict, sig_out);
    return DIL_OK;
  }
  if (s->svc_rc) return s->svc_rc;
  return s->svc_on ? DIL_ETIMEDOUT : DIL_EINVAL;
}

int dil_server_stop(dil_server *s) {
  if (!s) return DIL_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->svc_on) return sfail(s, DIL_EINVAL, "the interactive mode is not on");
    s->svc_stop = true;
  }
  s->cv_in.notify_all();
  s->svc.join();
  std::lock_guard<std::mutex> lk(s->mu);
  s->svc_on = false;
  s->cv_done.notify_all();
  return s->svc_rc;
}

}  // extern "C"
