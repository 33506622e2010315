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
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <thread>
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
  std::vector<uint32_t> req;  // request ids
  size_t m_pos = 0, m_len = 0, t_pos = 0, o_pos = 0, s_pos = 0;
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
  // statistics of the last run
  uint64_t batches = 0, overlapped = 0;
  double host_s = 0;
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
           dil_ctx_create(&ln.gctx[gi], device, 0) == DIL_OK && dil_ctx_set_mode(ln.gctx[gi], mode) == DIL_OK &&
           // a group call holds few tasks: four-wavefront workgroups give each
           // task 4 x 64 / l nonces per batch, so almost every task passes in
           // the first batch instead of needing a second or third
           (gi % 2 == 1 || dil_ctx_set_param(ln.gctx[gi], "persist.waves", 4) == DIL_OK);
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
  double host = 0;
  uint64_t batches = 0, overlapped = 0;
  uint32_t head = 0, done = 0;
  std::vector<Lane *> free_lanes;
  for (auto &ln : s->lanes) free_lanes.push_back(&ln);
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
      uint64_t t = now_ns();
      for (auto &g : ln.groups) {
        size_t ss = s->sig_bytes[g.li];
        for (size_t j = 0; j < g.req.size(); j++) {
          uint32_t r = g.req[j];
          done_ns[r] = t;
          if (g.op == 0) {
            memcpy(sig_out + sig_out_off[r], ln.h_sig + g.s_pos + j * ss, ss);
            verdict[r] = -1;
          } else {
            verdict[r] = ln.h_ver[g.t_pos + j];
          }
        }
        done += (uint32_t)g.req.size();
      }
      ln.busy = false;
      ln.groups.clear();
      free_lanes.push_back(&ln);
      progressed = true;
    }
    // admit
    uint64_t tnow = now_ns();
    uint32_t arrived = (uint32_t)(std::upper_bound(arrival_ns, arrival_ns + n, tnow) - arrival_ns);
    if (!free_lanes.empty() && head < arrived) {
      auto h0 = clk::now();
      Lane &ln = *free_lanes.back();
      size_t mbytes = 0;
      uint32_t per_group[NGROUP] = {};
      uint32_t end = head;
      while (end < arrived && end - head < s->max_batch) {
        size_t ml = msg_off[end + 1] - msg_off[end];
        const int gi = 2 * lv_index(level[end]) + op[end];
        // in arrival order: the first request whose group is full (its workspace
        // reservation) or whose message does not fit waits for the next batch
        if (per_group[gi] == s->group_cap || mbytes + ml > s->max_msg) break;
        per_group[gi]++;
        mbytes += ml;
        end++;
      }
      if (end > head) {
        free_lanes.pop_back();
        // group by (level, op) keeping arrival order within each group
        ln.groups.clear();
        for (int li = 0; li < NLV; li++)
          for (int o = 0; o < 2; o++) {
            Group g;
            g.li = li;
            g.op = o;
            for (uint32_t r = head; r < end; r++)
              if (lv_index(level[r]) == li && op[r] == o) g.req.push_back(r);
            if (!g.req.empty()) ln.groups.push_back(std::move(g));
          }
        size_t m_pos = 0, t_pos = 0, o_pos = 0, s_pos = 0;
        for (auto &g : ln.groups) {
          size_t ss = s->sig_bytes[g.li];
          g.m_pos = m_pos;
          g.t_pos = t_pos;
          g.o_pos = o_pos;
          g.s_pos = s_pos;
          uint64_t acc = 0;
          for (size_t j = 0; j < g.req.size(); j++) {
            uint32_t r = g.req[j];
            size_t ml = msg_off[r + 1] - msg_off[r];
            memcpy(ln.h_msg + m_pos + acc, msg + msg_off[r], ml);
            ln.h_off[o_pos + j] = acc;
            acc += ml;
            ln.h_key[t_pos + j] = key[r];
            if (g.op == 1) memcpy(ln.h_sig + s_pos + j * ss, sig_in + sig_in_off[r], ss);
          }
          ln.h_off[o_pos + g.req.size()] = acc;
          g.m_len = acc;
          m_pos += acc;
          t_pos += g.req.size();
          o_pos += g.req.size() + 1;
          s_pos += g.req.size() * ss;
        }
        bool ok = hipMemcpyAsync(ln.d_msg, ln.h_msg, std::max<size_t>(m_pos, 1), hipMemcpyHostToDevice, ln.st) ==
                      hipSuccess &&
                  hipMemcpyAsync(ln.d_off, ln.h_off, o_pos * 8, hipMemcpyHostToDevice, ln.st) == hipSuccess &&
                  hipMemcpyAsync(ln.d_key, ln.h_key, t_pos * 4, hipMemcpyHostToDevice, ln.st) == hipSuccess &&
                  (s_pos == 0 ||
                   hipMemcpyAsync(ln.d_sig, ln.h_sig, s_pos, hipMemcpyHostToDevice, ln.st) == hipSuccess);
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
        overlapped += others_busy ? 1 : 0;
        ln.busy = true;
        head = end;
        batches++;
        progressed = true;
        host += std::chrono::duration<double>(clk::now() - h0).count();
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
  s->batches = batches;
  s->overlapped = overlapped;
  s->host_s = host;
  return DIL_OK;
}

}  // extern "C"
