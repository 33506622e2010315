/*
 * libdil -- batched CRYSTALS-Dilithium (round-3 parameter sets 2, 3, 5, and
 * their FIPS 204 form ML-DSA-44 / 65 / 87) on AMD Instinct MI355X (gfx950).
 * C ABI.
 *
 * The operations are Dilithium.Gen, Dilithium.Sign (deterministic mode) and
 * Dilithium.Verify as given in Alg. 1, 2 and 3 of the paper, with the
 * parameter sets of its Tab. 1; one call processes a batch of independent
 * tasks (Sec. 3.1: one key generation, signing or verification is one task).
 * Byte layouts of keys and signatures follow the public round-3 (v3.1)
 * specification conventions, which the paper does not restate:
 *   level 2: pk 1312 B, sk 2528 B, signature 2420 B
 *   level 3: pk 1952 B, sk 4000 B, signature 3293 B
 *   level 5: pk 2592 B, sk 4864 B, signature 4595 B
 * Levels 44, 65 and 87 select ML-DSA-44 / 65 / 87 (FIPS 204, not covered by
 * the paper): the lattice parameters of levels 2 / 3 / 5 with a 64-byte tr, a
 * ctilde of 32 / 48 / 64 bytes that seeds SampleInBall whole, the key seed
 * H(xi || k || l), mu = H(tr || 0x00 || 0x00 || M) (pure signing, empty
 * context) and the mask seed rho'' = H(K || rnd || mu):
 *   level 44: pk 1312 B, sk 2560 B, signature 2420 B
 *   level 65: pk 1952 B, sk 4032 B, signature 3309 B
 *   level 87: pk 2592 B, sk 4896 B, signature 4627 B
 * Every batch, key-table and serving entry point takes all six levels;
 * dil_t0_ntt_batch (an ablation primitive) takes levels 2, 3, 5 only.
 *
 * Conventions for every batch entry point:
 *   - Buffer pointers are DEVICE pointers (hipMalloc'd or torch tensors on the
 *     same GPU as the context), owned by the caller; the library never frees
 *     or retains them after the call returns.
 *   - Row i of a fixed-stride array (keys, signatures) is task i's; message i
 *     is msg[msg_off[i] .. msg_off[i+1]) with msg_off holding count + 1
 *     uint64 entries on the device (lengths may be 0; any alignment).
 *   - key_idx may be NULL (task i uses key row i) or a device array of count
 *     uint32 key-row indices (resident key tables).  Every index must name a
 *     row of the key buffer: the batch entry points read the rows without
 *     bounds checks.  The key-table entry points check them on the device
 *     (see dil_sign_keyset).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *     Calls that finish synchronously say so.  Output i always belongs to
 *     input i, whatever order the device processes tasks in.
 *   - count == 0 is a no-op returning DIL_OK.
 *   - Errors are returned, never written into outputs:
 *       DIL_EINVAL  level not in {2,3,5,44,65,87}, NULL pointer with count > 0, bad mode;
 *       DIL_ENOMEM  the context cannot allocate its workspace;
 *       DIL_EHIP    a HIP launch/copy failed (dil_last_error() has the text);
 *       DIL_EMSG    a decreasing msg_off entry was found (detected on the
 *                   device; reported by calls that synchronise, and by
 *                   dil_ctx_check()); a key-table index outside its table
 *                   is reported the same way, as DIL_EINVAL;
 *       DIL_ETIMEDOUT  dil_server_wait ran out of time (the request stays
 *                   outstanding).
 *     A malformed signature is not an error: its verdict is 0 (Alg. 3).
 *   - One context serves one host thread at a time; calls that overlap on
 *     one context race on its workspace.
 */
#ifndef DIL_H
#define DIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIL_OK 0
#define DIL_EINVAL (-1)
#define DIL_ENOMEM (-2)
#define DIL_EHIP (-3)
#define DIL_EMSG (-4)
#define DIL_ETIMEDOUT (-5)

/* Execution forms for Sign (dil_ctx_set_mode):
 *   DIL_MODE_STAGED      one kernel launch per pipeline stage, host-driven
 *                        rejection loop over the still-active tasks (the host
 *                        synchronises once per loop round).
 *   DIL_MODE_PERSISTENT  fused persistent kernel with a device-side work queue
 *                        (asynchronous; no host round trips). */
#define DIL_MODE_STAGED 0
#define DIL_MODE_PERSISTENT 1

typedef struct dil_ctx dil_ctx;

/* Create a context on HIP device `device`.  workspace_bytes is a hint for the
 * initial workspace (0 = grow on demand).  Returns DIL_OK and *out, or an error. */
int dil_ctx_create(dil_ctx **out, int device, size_t workspace_bytes);
/* Release the context and its workspace (waits for its outstanding work). */
int dil_ctx_destroy(dil_ctx *ctx);
/* Select the Sign execution form (DIL_MODE_*). */
int dil_ctx_set_mode(dil_ctx *ctx, int mode);
/* Tuning knobs (0 = automatic):
 *   "persist.grid"  workgroups launched by the persistent Sign kernel;
 *   "persist.hmax"  tasks one workgroup holds at a time (1..slots per batch);
 *   "persist.waves" wavefronts per persistent workgroup: 1 (64 / l candidate
 *                   slots per batch), 2 or 4 (default; W * (64 / l) slots,
 *                   the challenge hashes on two lanes per slot); any other
 *                   value is DIL_EINVAL; the ML-DSA levels are built for 4
 *                   only (a persistent Sign call or dil_persist_capacity at
 *                   level 44 / 65 / 87 with 1 or 2 is DIL_EINVAL);
 *   "timing"        1 = record HIP events around the persistent Sign's setup
 *                   kernels and its loop kernel (read with dil_sign_timing);
 *   "graph"         1 = capture the launch sequences of persistent-mode Sign's
 *                   setup stages and of Verify into hipGraphs, replayed when a
 *                   call repeats the same level, buffers, count and schedule
 *                   (up to 16 graphs per context, least recently used
 *                   evicted; dropped when the workspace grows); the Sign loop
 *                   kernel, a single launch, is always launched directly;
 *   "ntt.variant"   form of dil_ntt_mul_batch, for the optimisation ablation
 *                   of the NTT primitive (Sec. 3.2, Sec. 4.2); every form
 *                   returns the same words: 0 (default) levels merged in
 *                   registers with one padded LDS transpose per transform,
 *                   1 the same transpose unpadded (bank conflicts), 2 one LDS
 *                   round trip per butterfly level, 3 unfused (forward NTT,
 *                   pointwise product and inverse NTT as three launches
 *                   through HBM, c used as the intermediate); other values
 *                   are DIL_EINVAL;
 *   "t0.variant"    form of dil_t0_ntt_batch, for the optimisation ablation
 *                   of the NTT(t0) stage of signing (Sec. 5, speedup
 *                   breakdown); every form returns the same words: 0
 *                   (default) unpacking merged into the NTT's registers,
 *                   padded LDS transpose (the Sign setup's code path), 1 the
 *                   same unpadded, 2 one fused kernel that stores t0 in HBM
 *                   and reads it back, 3 an unpacking kernel then an NTT
 *                   kernel through HBM; other values are DIL_EINVAL;
 *   "mldsa.internal" 0 (default) or 1: 1 makes the Sign and Verify calls of
 *                   the ML-DSA levels take formatted messages M' and hash
 *                   mu = H(tr || M') (FIPS 204's internal functions): the
 *                   caller builds M' = 0x00 || |ctx| || ctx || M for a
 *                   context string ctx (at most 255 bytes), or 0x01 || |ctx|
 *                   || ctx || OID || PH(M) for the pre-hash form; 0 hashes
 *                   tr || 0x00 || 0x00 || M (empty context).  A Sign or
 *                   Verify call at levels 2 / 3 / 5 with 1 fails with
 *                   DIL_EINVAL;
 *   "persist.tail"  slots per held task in the batches of a four-wavefront
 *                   workgroup once the work queue has run dry (rounded up to a
 *                   multiple of 4, at most the batch's slots): shorter last
 *                   batches, fewer speculative candidates; -1 (default) the
 *                   level's setting (20 at levels 2 / 44, 12 at 3 / 65, full
 *                   batches at 5 / 87), 0 full batches, 1..64 that many; a
 *                   value above 0 with another "persist.waves" or
 *                   "persist.pad" = 0 fails the Sign call with DIL_EINVAL;
 *                   the signatures do not depend on it;
 *   "persist.pad"   1 (default) or 0: 0 runs the four-wavefront Sign loop
 *                   kernel with every NTT / INTT transpose on the unpadded
 *                   (bank-conflicted) LDS layout, the padding step of the same
 *                   ablation inside the loop; the signatures are identical; a
 *                   persistent Sign call with 0 and another "persist.waves"
 *                   value, or at an ML-DSA level, fails with DIL_EINVAL. */
int dil_ctx_set_param(dil_ctx *ctx, const char *name, int64_t value);
/* Operations, for the workspace queries below. */
#define DIL_OP_KEYGEN 0
#define DIL_OP_SIGN 1
#define DIL_OP_VERIFY 2

/* Grow the context's workspace (synchronously) so that any call with up to
 * `count` tasks at `level` runs without allocating -- serving loops reserve the
 * largest batch they admit up front. */
int dil_ctx_reserve(dil_ctx *ctx, int level, uint32_t count);
/* As dil_ctx_reserve, for calls of one kind only: op (DIL_OP_*) at `level`,
 * against a resident key table (keyset != 0: A-hat and the NTT-domain secrets
 * come from the table and take no workspace) or not, in the context's current
 * Sign form and schedule knobs, with up to `count` tasks. */
int dil_ctx_reserve_call(dil_ctx *ctx, int level, int op, int keyset, uint32_t count);
/* Device bytes of workspace that one such call of exactly `count` tasks needs
 * (the same layout the call carves: per-task rows, plus the persistent Sign
 * kernel's per-workgroup scratch at the schedule that count gets).  Memory
 * budgets of serving loops are accounted with this figure.  The workspace is
 * allocated stream-ordered on the calling stream; growing it waits only for
 * this context's previous call. */
int dil_workspace_bytes(dil_ctx *ctx, int level, int op, int keyset, uint32_t count, size_t *bytes);
/* Synchronise `stream` and report, once, the conditions the device detected
 * since the last check: a decreasing msg_off entry (DIL_EMSG), a key-table
 * index outside its table (DIL_EINVAL) and Sign tasks dropped at the per-task
 * iteration limit, whose signature rows stay unwritten (DIL_EHIP; unreachable
 * in practice).  dil_last_error() names every condition that was set; all are
 * cleared. */
int dil_ctx_check(dil_ctx *ctx, void *stream);
/* Text of the last error on this context (static storage inside the context). */
const char *dil_last_error(dil_ctx *ctx);

/* Byte sizes for a level (Tab. 1 parameters, round-3 v3.1 layouts; FIPS 204 for 44 / 65 / 87). */
int dil_sizes(int level, size_t *pk_bytes, size_t *sk_bytes, size_t *sig_bytes);

/* Dilithium.Gen (Alg. 1) with caller-supplied 32-byte seeds zeta:
 * seeds[count][32] -> pk[count][PK], sk[count][SK].  (ML-DSA levels expand
 * H(xi || k || l) and store a 64-byte tr.) */
int dil_keygen_batch(dil_ctx *ctx, int level, const uint8_t *seeds, uint8_t *pk, uint8_t *sk, uint32_t count,
                     void *stream);

/* Dilithium.Sign (Alg. 2), deterministic (rho' = H(K || mu); ML-DSA levels:
 * rho'' = H(K || 0^32 || mu), FIPS 204's deterministic variant):
 * sk rows [n_keys][SK], messages (msg, msg_off), sig[count][SIG].
 * Output equals sequential Sign: the first kappa = 0, l, 2l, ... that passes
 * all four rejection checks.  In DIL_MODE_STAGED the call returns after the
 * batch has completed. */
int dil_sign_batch(dil_ctx *ctx, int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                   const uint64_t *msg_off, uint8_t *sig, uint32_t count, void *stream);

/* The randomized variant of round-3 Sign: as dil_sign_batch, but task i uses
 * rho' = rnd[64 i .. 64 i + 64) (caller-supplied random bytes, a device
 * buffer of count x 64 bytes, 4-byte aligned) instead of H(K || mu) (Alg. 2
 * computes rho' deterministically; every other step is the same).  At the
 * ML-DSA levels rnd holds 32 bytes per task (count x 32, 4-byte aligned) and
 * is hashed into the mask seed, rho'' = H(K || rnd[32 i .. 32 i + 32) || mu)
 * (FIPS 204's hedged signing).  rnd NULL is deterministic Sign.  DIL_EINVAL
 * for a misaligned rnd.  The caller owns the randomness: the output is a
 * deterministic function of (sk, M, rnd). */
int dil_sign_batch_rnd(dil_ctx *ctx, int level, const uint8_t *sk, const uint32_t *key_idx, const uint8_t *msg,
                       const uint64_t *msg_off, const uint8_t *rnd, uint8_t *sig, uint32_t count, void *stream);

/* Dilithium.Verify (Alg. 3) with strict signature decoding:
 * verdict[count] int32 = 1 accept, 0 reject. */
int dil_verify_batch(dil_ctx *ctx, int level, const uint8_t *pk, const uint32_t *key_idx, const uint8_t *msg,
                     const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count, void *stream);

/* ---- Resident key tables (serving) ----
 * A key table keeps n_keys key rows of one level on the device together with
 * what Sign and Verify would otherwise recompute per call: A-hat = ExpandA(rho)
 * (Alg. 1-3), NTT(s1), NTT(s2), NTT(t0) (Alg. 2) when secret keys are given,
 * NTT(t1 2^d) and tr = H(pk) (Alg. 3) when public keys are given.  pk and sk
 * are device arrays of n_keys rows (either may be NULL, not both; when both are
 * given row i of each must be one key pair).  The table owns copies of the rows
 * and may be used from any context on the same device, concurrently for
 * reads.  Creation is enqueued on `stream`. */
typedef struct dil_keyset dil_keyset;
int dil_keyset_create(dil_ctx *ctx, int level, const uint8_t *pk, const uint8_t *sk, uint32_t n_keys,
                      dil_keyset **out, void *stream);
/* Waits for the device, then frees the table. */
int dil_keyset_destroy(dil_keyset *ks);
/* Level, number of keys and device bytes held by the table (any pointer may be NULL). */
int dil_keyset_info(const dil_keyset *ks, int *level, uint32_t *n_keys, size_t *device_bytes);
/* dil_sign_batch / dil_verify_batch against a key table: task i uses key row
 * key_idx[i] (device array), or row i when key_idx is NULL.  Outputs are
 * identical to the batch entry points given the same key rows.  An index
 * outside the table is replaced by row 0 on the device before any key row is
 * read, and the error is reported as DIL_EINVAL by the next call that
 * synchronises (staged-mode Sign itself, or dil_ctx_check()). */
int dil_sign_keyset(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                    const uint64_t *msg_off, uint8_t *sig, uint32_t count, void *stream);
int dil_verify_keyset(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                      const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count, void *stream);

/* dil_verify_keyset for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and outputs, with the call's workspace in a fixed device
 * array of 16 MiB that the library holds on every GPU it runs on until the
 * process ends, instead of the context's pool; the call allocates nothing and
 * enqueues only kernels on `stream` (no memset, no side stream).  count is
 * limited by that array: 11,847 tasks at level 2 or 44, 11,335 at level 3
 * or 65, 9,320 at level 5 or 87; a larger count is DIL_EINVAL with the limit in
 * dil_last_error().  The context supplies the device and the error words
 * (dil_ctx_check reports a key index outside the table, as for
 * dil_verify_keyset).  All calls on one
 * GPU share the array: calls that overlap on one GPU (other streams, other
 * threads, other contexts) race on it and must be ordered by the caller. */
int dil_verify_keyset_noalloc(dil_ctx *ctx, const dil_keyset *ks, const uint32_t *key_idx, const uint8_t *msg,
                              const uint64_t *msg_off, const uint8_t *sig, int32_t *verdict, uint32_t count,
                              void *stream);

/* ---- Continuous-batching serving engine ----
 * Host-side dispatcher over key tables (at most one per level, any of the six
 * levels; a level without a table is not served).  It keeps up to n_streams batches in flight, each on its own HIP
 * stream with its own contexts; whenever a stream is free it admits the
 * requests that have arrived, in arrival order, splits the batch by
 * (level, op) into dil_sign_keyset / dil_verify_keyset calls, and stages
 * messages, key indices and signatures through pinned buffers (max_msg_bytes
 * of message data per batch, at most max_batch requests).
 * Device memory: at creation each stream reserves, for every (level, op)
 * group, the workspace of a call of C requests (dil_workspace_bytes), where C
 * (at most max_batch) is the largest count for which all streams' workspaces
 * and device staging buffers fit mem_budget bytes; DIL_ENOMEM if not even
 * C = 1 fits.  A batch then holds at most C requests of each group: a request
 * that would exceed its group's C (or the message buffer) waits for the next
 * batch, it never fails, and no call allocates while serving.
 * The (level, op) groups of a batch run concurrently, each on a stream and
 * context of its own; that needs more hardware queues than HIP's default of 4
 * per process, so the process should set GPU_MAX_HW_QUEUES (e.g. 16) before
 * HIP starts.  mode is DIL_MODE_STAGED or DIL_MODE_PERSISTENT for Sign; the
 * persistent Sign calls use four-wavefront workgroups ("persist.waves" = 4).
 * mode | DIL_SERVER_MLDSA_INTERNAL: the requests of the ML-DSA levels carry
 * formatted messages M' ("mldsa.internal" = 1 on those groups: context
 * strings, pre-hashed messages); round-3 requests are unaffected.  Other mode
 * bits give DIL_EINVAL. */
#define DIL_SERVER_MLDSA_INTERNAL 0x100
typedef struct dil_server dil_server;
/* tables: n_tables key tables (host array of handles), each level at most
 * once (a table's level comes from the table); DIL_EINVAL otherwise. */
int dil_server_create_tables(dil_server **out, int device, dil_keyset *const *tables, int n_tables, int n_streams,
                             uint32_t max_batch, size_t max_msg_bytes, size_t mem_budget, int mode);
/* The same with the round-3 tables passed by level (ks2 / ks3 / ks5, each
 * may be NULL). */
int dil_server_create(dil_server **out, int device, dil_keyset *ks2, dil_keyset *ks3, dil_keyset *ks5,
                      int n_streams, uint32_t max_batch, size_t max_msg_bytes, size_t mem_budget, int mode);
/* Waits for the device and frees the engine (not the key tables). */
int dil_server_destroy(dil_server *s);
const char *dil_server_last_error(dil_server *s);
/* Statistics (any pointer may be NULL): batches launched in the last run, of
 * them those launched while another batch was still in flight, host seconds
 * spent forming and launching them; and the per-group request cap C and the
 * device bytes the engine reserved under its memory budget. */
int dil_server_stats(dil_server *s, uint64_t *batches, double *host_seconds, uint64_t *overlapped,
                     uint32_t *group_cap, size_t *reserved_bytes);
int dil_server_run(dil_server *s, uint32_t n, const uint8_t *op, const uint8_t *level, const uint32_t *key,
                   const uint8_t *msg, const uint64_t *msg_off, const uint8_t *sig_in, const uint64_t *sig_in_off,
                   const uint64_t *arrival_ns, uint8_t *sig_out, const uint64_t *sig_out_off, int32_t *verdict,
                   uint64_t *done_ns);

/* Interactive mode of the same engine (continuous batching of requests that
 * application threads submit one by one; the spec serving loop, not in
 * the paper).  dil_server_start starts a dispatcher thread that forms batches
 * as streams free up, under the admission rules above (requests in
 * submission order, at most the group cap per (level, op), messages within
 * max_msg_bytes), so that requests submitted while earlier batches run join
 * the next one.  dil_server_run returns DIL_EINVAL while the mode is on.
 * All buffers are host memory owned by the caller; the engine copies what it
 * needs before dil_server_submit returns.  Thread-safe: any host thread may
 * submit, poll and wait at once (start / stop / destroy from one thread).
 *
 * dil_server_submit: op 0 = Sign, 1 = Verify of msg[0 .. msg_len) with row
 *   `key` of the level's key table; sig (Verify only) holds the level's
 *   signature size (dil_sizes).  Writes a ticket.  DIL_EINVAL for an unknown
 *   level or op, a key row outside its table, a message longer than
 *   max_msg_bytes, a NULL pointer, or when the mode is off or stopping; the
 *   dispatcher's error code once it has failed.
 * dil_server_poll: *done = 1 and the result (Sign: the signature in sig_out,
 *   *verdict = -1; Verify: *verdict = 1 accept / 0 reject) once the request
 *   has finished, else *done = 0.  A result is handed out once; a ticket not
 *   outstanding (unknown, or already handed out) gives DIL_EINVAL.
 * dil_server_wait: as poll, blocking up to timeout_ms (< 0: no limit);
 *   DIL_ETIMEDOUT if the request is still running then.
 * dil_server_stop: finishes every submitted request, then stops the
 *   dispatcher; results not yet collected stay available to poll / wait.
 * A device failure or a batch with no progress for 60 s stops the
 *   dispatcher; every later call returns its error (dil_server_last_error
 *   has the text).  dil_server_stats counts the batches since start. */
int dil_server_start(dil_server *s);
int dil_server_submit(dil_server *s, int op, int level, uint32_t key, const uint8_t *msg, uint64_t msg_len,
                      const uint8_t *sig, uint64_t *ticket);
int dil_server_poll(dil_server *s, uint64_t ticket, int *done, int32_t *verdict, uint8_t *sig_out);
int dil_server_wait(dil_server *s, uint64_t ticket, int32_t timeout_ms, int32_t *verdict, uint8_t *sig_out);
int dil_server_stop(dil_server *s);

/* Number of Sign loop iterations (candidate signatures) the last dil_sign_batch
 * on this context evaluated in total, and the number the sequential algorithm
 * needs (sum over tasks of the winning iteration index + 1).  Synchronises. */
int dil_sign_stats(dil_ctx *ctx, uint64_t *evaluated, uint64_t *sequential);

/* For the context's current "persist.waves" shape W: workgroups of the
 * persistent Sign kernel the device keeps resident at once, and candidate
 * slots per workgroup batch (W * (64 / l)), for schedule tuning. */
int dil_persist_capacity(dil_ctx *ctx, int level, int *resident_groups, int *slots_per_batch);

/* Event-measured durations (ms) of the most recent persistent dil_sign_batch
 * calls made since the "timing" parameter was set (at most 64 are kept):
 * setup kernels (mu, rho', ExpandA, secret NTTs) and the persistent
 * rejection-loop kernel, oldest first.  Fills at most max_calls entries of
 * each caller-owned array (either may be NULL), stores the number filled in
 * *n_calls, and synchronises on the recorded events. */
int dil_sign_timing(dil_ctx *ctx, float *setup_ms, float *loop_ms, int max_calls, int *n_calls);

/* Primitive: c_i = INTT(NTT(a_i) o b_i) for count polynomials of 256
 * coefficients (Sec. 2.2), a and b canonical int32 in [0, q), b read as
 * NTT-domain values (slot j = evaluation at psi^(2 brv8(j)+1), psi = 1753);
 * c canonical.  Uses Montgomery arithmetic internally.  a, b and c must be
 * 16-byte aligned (DIL_EINVAL otherwise) and c must not overlap a or b. */
int dil_ntt_mul_batch(dil_ctx *ctx, const int32_t *a, const int32_t *b, int32_t *c, uint64_t count, void *stream);

/* Primitive: ExpandA rejection sampling (Sec. 2.3, Sec. 3.4) of count
 * polynomials from 34-byte inputs seeds[count][34] (SHAKE128, 3 bytes ->
 * 23-bit candidate, kept if < q) -> out[count][256] canonical int32.
 * count must be below 2^32 (DIL_EINVAL otherwise). */
int dil_expand_a_batch(dil_ctx *ctx, const uint8_t *seeds34, int32_t *out, uint64_t count, void *stream);

/* Stage of signing: t0-hat = NTT(t0) with t0 unpacked from each secret key
 * (Alg. 2 precomputes NTT(t0); Sec. 5 uses this stage for its speedup
 * breakdown), in the form "t0.variant" selects.  sk[count][SK] (rows of
 * dil_sizes' sk bytes, 8-byte aligned) -> t0_hat[count][k][256] int32
 * reduced to [0, q), natural NTT slot order (16-byte aligned; forms 2 and 3
 * also use it as their intermediate).  Device buffers owned by the caller;
 * asynchronous on `stream`; DIL_EINVAL for a bad level, null or misaligned
 * buffers; count = 0 is a no-op. */
int dil_t0_ntt_batch(dil_ctx *ctx, int level, const uint8_t *sk, int32_t *t0_hat, uint32_t count, void *stream);

/* Diagnostic: the vector-ALU issue-rate probe behind the benchmark's peak.
 * Launches `groups` workgroups of 256 lanes; every lane executes iters x 128
 * instructions of one kind (0 v_xor_b32, 1 v_add_u32, 2 v_bitop3_b32,
 * 3 v_alignbit_b32, 4 v_mul_lo_u32, 5 v_mad_u64_u32) in eight independent
 * dependency chains and stores one word to out[groups * 256] (device).
 * *instructions (optional) receives the lane-instructions the launch
 * executes; dividing by its event-timed duration gives lane-ops/s. */
int dil_alu_probe(dil_ctx *ctx, int kind, uint32_t iters, uint32_t groups, uint32_t *out, void *stream,
                  uint64_t *instructions);

#ifdef __cplusplus
}
#endif
#endif
