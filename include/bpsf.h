/*
 * bpsf.h - C ABI of the MI355X (gfx950) BP-SF decoder library (libbpsf.so).
 *
 * BP-SF ("Fully Parallelized BP Decoding for Quantum LDPC Codes Can
 * Outperform BP-OSD", arXiv 2507.00254) decodes a syndrome s of a binary
 * parity-check matrix H (the decoding problem of Section II-B: find e with
 * e H^T = s) in three steps (Algorithm 1):
 *   1. flooding normalized min-sum BP (Section II-B, steps 1-4, Eq. (c2v))
 *      while counting how often every hard decision flips;
 *   2. if BP does not reproduce s within max_iter iterations, take the k
 *      most-flipped bits Phi and form trial vectors t over Phi;
 *   3. decode every trial syndrome s' = s + t H^T with an independent short
 *      BP and return e' + t for a successful trial (the lightest one, or the
 *      lowest-index one, see bpsf_params.select_mode).
 *
 * Conventions for every entry point:
 *   - return 0 on success or a negative BPSF_E* code; bpsf_last_error() then
 *     returns a message for the calling thread; nothing else reports errors
 *     and no C++ exception crosses the ABI;
 *   - "device" pointers are HIP device memory of the current device, "host"
 *     pointers are ordinary host memory; every buffer is owned by the caller
 *     and must stay valid until the work enqueued on `stream` has completed;
 *   - `stream` is a hipStream_t (NULL = the default stream); decoding is
 *     asynchronous on that stream and outputs are valid once it synchronizes;
 *   - a code handle owns device copies of the code tables and a scratch area
 *     reused by every decode call on it: calls on one handle must be issued
 *     on one stream (or otherwise ordered); handles are independent.
 */
#ifndef BPSF_H
#define BPSF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BPSF_OK 0
#define BPSF_EINVAL (-1)   /* bad shape, pointer or parameter */
#define BPSF_ENOMEM (-2)   /* device memory allocation failed */
#define BPSF_ENOTSUP (-3)  /* the code's shape has no compiled kernel tile */
#define BPSF_EDEVICE (-4)  /* a HIP call failed */

/* Trial vector sets (Algorithm 1, combinations(Phi, w_max)). */
#define BPSF_TRIALS_ALL_SUBSETS 0   /* all 2^k subsets of Phi; trial index = mask, bit j <-> Phi[j] */
#define BPSF_TRIALS_WEIGHT_LE 1     /* subsets of weight 1..w_max, by weight, then combination order */
#define BPSF_TRIALS_TABLE 2         /* the caller's list (bpsf_set_trial_table), e.g. n_s sampled
                                       subsets per weight 1..w_max as in Section IV */

/* Result selection among successful trials (Section IV). */
#define BPSF_SELECT_MIN_WEIGHT 0    /* lightest e' + t; ties to the lower trial index */
#define BPSF_SELECT_FIRST 1         /* lowest successful trial index */

/* bpsf_params.flags (test and study options) */
#define BPSF_FLAG_NO_EARLY_STOP 1   /* run max_iter iterations even after e H^T = s */
#define BPSF_FLAG_FORCE_PP 2        /* run the trials even when the first BP succeeded */
#define BPSF_FLAG_PRUNE 4           /* with BPSF_SELECT_FIRST only: a trial is skipped, or stopped,
                                       once a lower-index trial of its shot has succeeded (the
                                       result is the same; fewer trial iterations run) */
#define BPSF_FLAG_LAYERED 8         /* layered BP schedule instead of flooding, for every BP of the
                                       call (Section V runs the [[288,12,18]] circuit-level decoders
                                       with it, Fig. 288_circ): the checks are
                                       coloured greedily in index order (each takes the smallest
                                       layer unused by an earlier check sharing a bit) and visited
                                       by layer, then index; each check turns the posteriors of its
                                       bits, less its previous c2v, into v2c, applies Eq. (c2v) and
                                       adds the new c2v back. Single-code calls on one-wave codes
                                       only (BPSF_ENOTSUP for the irregular-code families, mixed
                                       calls, the server) */

#define BPSF_PREC_FP32 0            /* messages in float */
#define BPSF_PREC_FP64 1            /* messages in double */

typedef struct bpsf_code_s* bpsf_code;

typedef struct {
  int32_t max_iter;       /* i_max of the first BP, 1..255 */
  int32_t cand_max_iter;  /* i_max of every trial BP, 1..4095 */
  int32_t k;              /* |Phi|, 0..16; 0 = plain BP (no trials); with BPSF_TRIALS_TABLE up to
                             32 on codes of the sparse family, 64 with a 64-bit list
                             (bpsf_set_trial_table64; Section V's complexity study uses 50) */
  int32_t cand_mode;      /* BPSF_TRIALS_* */
  int32_t w_max;          /* BPSF_TRIALS_WEIGHT_LE: largest trial weight, 1..k */
  int32_t select_mode;    /* BPSF_SELECT_* */
  double alpha;           /* > 0: fixed normalization of c2v (e.g. 0.625); 0: alpha_i = 1 - 2^-i */
  int32_t flags;          /* BPSF_FLAG_* */
  int32_t precision;      /* BPSF_PREC_* */
} bpsf_params;

typedef struct {
  int64_t main_iterations;   /* first-BP iterations summed over the shots of the last call */
  int64_t trial_iterations;  /* trial-BP iterations summed over every trial run; with
                                BPSF_TRIALS_ALL_SUBSETS the empty trial of a failed shot is
                                not run (it would repeat the first cand_max_iter iterations of
                                the failed first BP) unless FORCE_PP or NO_EARLY_STOP is set
                                or cand_max_iter > max_iter */
  int64_t rerun_iterations;  /* iterations of the re-runs that emit winning trials; in calls of
                                the one-wave and sparse families (bpsf_decode, bpsf_mix_* calls of
                                at most 65536 shots, the request loop's batches) the trials of the
                                first failed shots (as many as 256 MiB of kept corrections cover,
                                4 B per lane of a decode per trial and code; 1 MiB per batch of the
                                request loop) keep their corrections and their winners are copied,
                                not re-run; the wide family, larger mixed calls and
                                bpsf_decode_noalloc re-run every winner */
  int64_t failed_shots;      /* shots whose first BP failed (or all shots with FORCE_PP, k > 0) */
  int64_t converged_trials;  /* trials that reproduced their syndrome */
  int64_t errors;            /* internal consistency failures (must be 0) */
} bpsf_stats;

/*
 * Load a parity-check matrix H (M x N, entries 0/1) given by rows:
 * row_ptr[M+1] and col_idx[row_ptr[M]] (host, int32; column indices of each
 * row strictly ascending and in [0, N)). The Tanner graph is the bipartite
 * graph of H (Section II-B): bits are columns, checks are rows. Builds the
 * device tables (edge layouts) on the current device; *out receives a handle
 * to free with bpsf_free_code. Fails with BPSF_ENOTSUP when the row and column
 * weights have no compiled kernel family: currently regular codes with row
 * weight 6 and column weight 3 of up to 576 checks and 1152 bits (the
 * bivariate-bicycle and coprime-BB codes of Appendix A), and with row weight
 * 10 and column weight 5 of up to 576 checks and 576 bits (the
 * generalized-bicycle code of Appendix A); otherwise, codes whose rows have
 * weight 2..8 and columns weight at most 3 (irregular weights allowed) of up
 * to 960 checks and 2688 bits run one decode per workgroup of three waves
 * (e.g. the phenomenological matrix of [[144,12,12]] over 12 rounds; float
 * messages, and double where the device gives a workgroup enough LDS, else
 * bpsf_decode fails with BPSF_ENOTSUP); otherwise, codes with rows of weight
 * 2..48 and columns of weight at most 10 of up to 1024 checks and 9216 bits
 * whose edges fit one workgroup's LDS as floats (4 B per edge: about 39,000
 * edges) run one decode per workgroup of sixteen waves (e.g. the circuit-level
 * detector error model of [[144,12,12]] over 12 rounds, Section V-B; float
 * messages only, double fails with BPSF_ENOTSUP). Codes of these two last
 * kinds do not mix with others (bpsf_mix_create), take only the flooding
 * schedule, and have no per-iteration trace or tunable launch shape.
 */
int bpsf_load_code(const int32_t* row_ptr, const int32_t* col_idx, int32_t M, int32_t N, bpsf_code* out);

/* Release a handle and its device memory (NULL is ignored). Synchronizes the device. */
void bpsf_free_code(bpsf_code code);

/*
 * Decode `shots` syndromes.
 *   syndromes   device, uint8 [shots][M], each entry 0 or 1 (only bit 0 is read)
 *   priors      host, double [N], error probability p_v of every bit, each in
 *               (0, 1); channel LLR l_v = log((1 - p_v) / p_v) (Section II-B
 *               step 1) is computed on the host in double and cached on the
 *               device for the next call with the same priors; a call whose
 *               priors differ from the handle's last ones (or whose trial set
 *               differs) first waits for the work already enqueued on
 *               `stream`, which may still read the old tables
 *   params      host; see bpsf_params
 *   corrections device, uint8 [shots][N]: the estimate e (0/1); when no trial
 *               succeeds it is the first BP's last hard decision
 *   converged   device, uint8 [shots]: 1 iff corrections[i] H^T = s_i
 *   iterations  device, int32 [shots]: first-BP iterations, plus the winning
 *               trial's iterations when a trial produced the result
 *   stream      hipStream_t
 * shots may be 0. Scratch grows with the largest shot count seen and is
 * reused; the call allocates device memory only when it must grow.
 */
int bpsf_decode(bpsf_code code, const uint8_t* syndromes, const double* priors, int64_t shots,
                const bpsf_params* params, uint8_t* corrections, uint8_t* converged, int32_t* iterations,
                void* stream);

/*
 * bpsf_decode for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and work counters as bpsf_decode, but the call's
 * scratch (work counters, one 64-bit trial key and one failure record per
 * shot) lives in a fixed array of 32 MiB that the library holds on every
 * device it runs on until the process ends, and the call allocates nothing
 * (the code's own tables are sized when it is loaded). The current device
 * must be the code's. Calls needing more scratch than the array holds
 * (8 + 4 * record words bytes per shot, e.g. 272 bytes per shot of
 * [[144,12,12]] with |Phi| = 6 in large calls, 944 bytes in calls of at most
 * 8192 shots, which run a kernel family with longer records) fail with
 * BPSF_EINVAL and enqueue nothing. Every such call on one device shares
 * that device's array: calls whose work overlaps on the device (other
 * streams, other threads, other handles) race and must be ordered by the
 * caller; bpsf_last_stats reports the last call's counters until the next
 * such call on the device.
 */
int bpsf_decode_noalloc(bpsf_code code, const uint8_t* syndromes, const double* priors, int64_t shots,
                        const bpsf_params* params, uint8_t* corrections, uint8_t* converged, int32_t* iterations,
                        void* stream);

/*
 * Grow the handle's scratch now for calls of up to `shots` shots with these
 * parameters (their k and the launch shape set the record size; every shape
 * a call of up to `shots` shots can take is covered, the small family's
 * longer records included), so that such calls allocate nothing: for
 * callers that cannot allocate later, e.g. under HIP graph capture or in a
 * serving loop. Synchronous.
 */
int bpsf_reserve(bpsf_code code, int64_t shots, const bpsf_params* params);

/* Work counters of the last bpsf_decode on `code` (host out). Waits for `stream`. */
int bpsf_last_stats(bpsf_code code, void* stream, bpsf_stats* out);

/*
 * Debug entry point: plain BP (no trials) on one syndrome, recording every
 * iteration. syndrome host uint8 [M]; priors host double [N]; params as for
 * bpsf_decode (k, cand_* ignored). lout_trace host Real [max_iter][N] and
 * c2v_trace host Real [max_iter][M*W] (Real = float or double by
 * params->precision; c2v in row order of H, W = row weight) may be NULL.
 * hard_out host uint8 [N]; *iters_out, *converged_out as for bpsf_decode.
 * Synchronous; allocates and frees its own device buffers.
 */
int bpsf_bp_trace(bpsf_code code, const uint8_t* syndrome, const double* priors, const bpsf_params* params,
                  void* lout_trace, void* c2v_trace, uint8_t* hard_out, int32_t* iters_out,
                  uint8_t* converged_out);

/*
 * Trial vectors the parameters produce (host only, no device needed): returns
 * their number n (or a negative BPSF_E* code) and, when masks_out is not NULL,
 * writes min(n, cap) k-bit masks in trial order (bit j <-> Phi[j], Phi[0] the
 * most-flipped bit) to the host array masks_out.
 */
int64_t bpsf_num_trials(const bpsf_params* params, uint32_t* masks_out, int64_t cap);

/*
 * Per-phase timing. With enable != 0, every later bpsf_decode on this handle
 * records HIP events on its stream around each of its kernels (the events are
 * created here, once). bpsf_last_timing waits for the last decode's stream and
 * writes ms_out[4] = {whole call, first BP, trial BPs, winner re-runs}
 * (host out; phases that did not run report 0).
 */
int bpsf_set_timing(bpsf_code code, int enable);
int bpsf_last_timing(bpsf_code code, float* ms_out);

/*
 * Decoding shots of several codes in one go. A mix handle names up to 8
 * loaded codes (distinct handles on one device that share a kernel family:
 * equal row and column weights, as the bivariate-bicycle codes of Appendix A
 * do; otherwise BPSF_ENOTSUP). It owns a scratch area of its own; the codes
 * must outlive it and keep their tables, but their LLR and trial tables are
 * refreshed by every bpsf_mix_decode, so calls on a mix and on its codes must
 * be ordered (one stream). bpsf_mix_free waits for the device.
 */
typedef struct bpsf_mix_s* bpsf_mix;
int bpsf_mix_create(const bpsf_code* codes, int32_t n_codes, bpsf_mix* out);
void bpsf_mix_free(bpsf_mix mix);

/*
 * Decode `shots` shots, shot i being a syndrome of codes[shot_code[i]]. Every
 * decode phase of Algorithm 1 (first BP, trial BPs, re-runs of the winners)
 * is one persistent launch over all codes: a wave takes decodes of one code
 * at a time and moves to another code once that one's work is taken, so the
 * codes share one tail instead of one each. Each shot's result is what
 * bpsf_decode returns for it alone with the same priors and parameters.
 *   shot_code    device, int32 [shots], entries in [0, n_codes); shots with
 *                other entries are skipped (outputs untouched) and counted
 *                in bpsf_mix_last_stats's *invalid_shots
 *   syndromes    device, uint8 [shots][syn_stride]; row i holds s_i in its
 *                first M bytes of its code (syn_stride >= every M)
 *   priors       host, priors[c] -> double [N of code c], as for bpsf_decode
 *   params       host, shared by every code
 *   corrections  device, uint8 [shots][corr_stride]; the first N bytes of
 *                row i are written (corr_stride >= every N)
 *   converged, iterations   device [shots], as for bpsf_decode
 * Scratch: 8 * n_codes + 4 + 4 * (rec words) bytes per shot, grown as
 * needed and reused.
 */
int bpsf_mix_decode(bpsf_mix mix, const int32_t* shot_code, const uint8_t* syndromes, int64_t syn_stride,
                    const double* const* priors, int64_t shots, const bpsf_params* params,
                    uint8_t* corrections, int64_t corr_stride, uint8_t* converged, int32_t* iterations,
                    void* stream);

/* bpsf_reserve for a mix: its scratch for calls of up to `shots` shots. */
int bpsf_mix_reserve(bpsf_mix mix, int64_t shots, const bpsf_params* params);

/*
 * As bpsf_mix_decode, with the shots grouped by code instead of listed:
 * counts (host int64 [n_codes]) gives each code's number of shots, and code
 * c's shots are the counts[c] rows following those of codes 0..c-1 (no
 * device-side grouping pass; shots = the sum of counts).
 */
int bpsf_mix_decode_grouped(bpsf_mix mix, const int64_t* counts, const uint8_t* syndromes, int64_t syn_stride,
                            const double* const* priors, const bpsf_params* params, uint8_t* corrections,
                            int64_t corr_stride, uint8_t* converged, int32_t* iterations, void* stream);

/* Work counters of the last bpsf_mix_decode, per code (host out [n_codes]),
 * and the number of shots whose code index was out of range (may be NULL).
 * Waits for `stream`. */
int bpsf_mix_last_stats(bpsf_mix mix, void* stream, bpsf_stats* per_code, int64_t* invalid_shots);

/*
 * Launch shape. A decode kernel runs D decodes per wavefront ("decodes per
 * wave", a power of two; 64 / D lanes per decode) in a persistent grid of
 * W waves per compute unit. Results do not depend on either, nor on the
 * kernel family: row-weight-6 codes have a large family and a small one
 * with a third of the checks and bits per lane. A bpsf_decode call of at
 * most 4096 x D shots, D being the small family's largest decodes per wave
 * for the code (8192 shots for [[144,12,12]]), or any call once D is fixed,
 * runs the family with the fewest items per lane that fits (at D); a larger
 * call runs the large family at its largest D (small calls leave the GPU
 * mostly idle, so one iteration of one wave is their latency). Mixed calls
 * follow the same rule at 2048 x D shots when every code takes the same
 * family.
 * bpsf_tile_options writes the D values the code fits, most first, to host
 * d_out (up to cap) and returns their number. bpsf_set_tile fixes D and W
 * for later calls on the handle (0 = default: as above, as many waves as
 * fit). bpsf_autotune times bpsf_decode on a sample (device
 * syndromes [shots][M], host priors, as for bpsf_decode; best of `reps`
 * calls after one untimed call) for every D and a range of W, keeps the
 * fastest on the handle and describes it in *out (host). It allocates and
 * frees output buffers for the sample and synchronizes `stream`.
 */
typedef struct {
  int32_t decodes_per_wave;  /* D chosen */
  int32_t waves_per_cu;      /* W chosen */
  float ms;                  /* its time on the sample */
  int32_t candidates;        /* (D, W) pairs timed */
} bpsf_tuning;
int bpsf_tile_options(bpsf_code code, int32_t* d_out, int32_t cap);
int bpsf_set_tile(bpsf_code code, int32_t decodes_per_wave, int32_t waves_per_cu);
int bpsf_autotune(bpsf_code code, const uint8_t* syndromes, const double* priors, int64_t shots,
                  const bpsf_params* params, int32_t reps, void* stream, bpsf_tuning* out);

/*
 * Request loop (the serving counterpart of the paper's parallel CPU
 * implementation, Section VI, which feeds syndromes through input and output
 * queues). A server decodes requests (a batch of host syndromes of one of
 * its codes) as they arrive, on a worker thread of its own. Codes (up to 8,
 * one kernel family when batching), their priors (host double [N] each,
 * copied) and the parameters are fixed at creation.
 *
 * Device memory: one pool per server of device_budget_bytes (0: half the
 * device memory free at creation as reported by hipMemGetInfo, at most what
 * every lane needs for a batch of max_batch_shots), allocated at creation.
 * A batch of n shots takes a region of n * (max M + max N + 5) bytes (plus
 * alignment) and, when batching, the scratch of its decode; the region
 * returns to the pool when the batch completes. A request fails at submit
 * (BPSF_EINVAL) only when it is larger than max_batch_shots or than the
 * whole pool can hold (bpsf_server_memory reports that size); otherwise it
 * waits until a lane and enough pool memory are free.
 *   batching = 1: continuous batching over `lanes` (1..8) streams. Whenever a
 *     lane is free, the waiting requests, in arrival order, that fit in
 *     max_batch_shots and in a free region of the pool are admitted into
 *     one batch: copied to the device grouped by code, decoded by one mixed
 *     decode (as bpsf_mix_decode_grouped), copied back in one transfer.
 *     Requests that arrive while batches run wait for the next free lane,
 *     so batches overlap on the device.
 *   batching = 0: each request decoded alone with bpsf_decode on its code,
 *     in arrival order, one at a time (lanes must be 1): the per-request form.
 * Pinned host memory per lane: max_batch_shots * (max M + max N + 5) bytes.
 * Creation runs every kernel shape the server can launch once, on zero
 * syndromes (first launches load code and would add milliseconds to a
 * request). Results are what bpsf_decode returns for each shot alone.
 * bpsf_server_submit enqueues a request (host syndromes uint8 [n][M of the
 * code]; outputs host corrections uint8 [n][N], converged uint8 [n],
 * iterations int32 [n]; all must stay valid until the request is collected)
 * and writes its id. bpsf_server_wait blocks until request `id` is done,
 * collects it (the id is then unknown) and writes its latency from submission
 * in seconds (may be NULL). bpsf_server_poll writes up to cap ids of requests
 * completed since the last poll (host int64 out) and returns their number.
 * bpsf_server_replay is an open-loop load driver on the calling thread:
 * request i (code[i], shots[i], host buffers as for submit) is submitted
 * arrival_s[i] seconds after the start (non-decreasing), whatever is still in
 * flight; once all are done it collects them and writes latency_s[i] =
 * completion - scheduled arrival and *wall_s (may be NULL) = the time from
 * the start to the last completion. bpsf_server_counters reports batches
 * launched, shots they held and requests completed. bpsf_server_memory
 * reports the pool size, the bytes in use now and at most since creation
 * (warm-up excluded), the largest request the pool can hold, and how many
 * requests had to wait for pool memory (host outs, any may be NULL).
 * bpsf_server_destroy finishes the queued work and frees the server; it
 * returns the first error the worker met, if any.
 */
typedef struct bpsf_server_s* bpsf_server;
int bpsf_server_create(const bpsf_code* codes, int32_t n_codes, const double* const* priors,
                       const bpsf_params* params, int32_t lanes, int64_t max_batch_shots, int32_t batching,
                       int64_t device_budget_bytes, bpsf_server* out);
int bpsf_server_submit(bpsf_server server, int32_t code, const uint8_t* syndromes, int32_t n,
                       uint8_t* corrections, uint8_t* converged, int32_t* iterations, int64_t* id_out);
int bpsf_server_wait(bpsf_server server, int64_t id, double* latency_s_out);
int64_t bpsf_server_poll(bpsf_server server, int64_t* ids_out, int64_t cap);
int bpsf_server_replay(bpsf_server server, int64_t n_requests, const double* arrival_s, const int32_t* code,
                       const int32_t* shots, const uint8_t* const* syndromes, uint8_t* const* corrections,
                       uint8_t* const* converged, int32_t* const* iterations, double* latency_s,
                       double* wall_s);
int bpsf_server_counters(bpsf_server server, int64_t* batches, int64_t* batch_shots, int64_t* requests_done);
int bpsf_server_memory(bpsf_server server, int64_t* budget, int64_t* in_use, int64_t* peak, int64_t* max_request,
                       int64_t* waited_for_memory);
int bpsf_server_destroy(bpsf_server server);

/*
 * Trial list for params.cand_mode = BPSF_TRIALS_TABLE on this handle:
 * masks (device uint32, owned by the caller, valid while such decodes run)
 * holds n_trials (1..2^31-1) k-bit masks in trial order, bit j <-> Phi[j]
 * (bits at or above k are ignored); shot i uses masks[i * stride + t], so
 * stride 0 gives every shot the same list and stride n_trials one list per
 * shot (in a mixed call i is the shot's row in the call). masks = NULL
 * clears the list. Takes effect on later calls.
 */
int bpsf_set_trial_table(bpsf_code code, const uint32_t* masks, int64_t n_trials, int64_t stride);

/*
 * The same with 64-bit masks (device uint64), for |Phi| up to 64 on codes of
 * the sparse family (the circuit-level matrices); other codes then fail with
 * BPSF_ENOTSUP at decode time when k > 16. Replaces any 32-bit list.
 */
int bpsf_set_trial_table64(bpsf_code code, const uint64_t* masks, int64_t n_trials, int64_t stride);

/* Shape of a loaded code: M, N, edges, row weight, column weight (host outs, any may be NULL). */
int bpsf_code_info(bpsf_code code, int32_t* M, int32_t* N, int32_t* edges, int32_t* row_weight,
                   int32_t* col_weight);

/*
 * The LDS layout that bpsf_load_code gives a code of the sparse family (the
 * large irregular matrices, such as circuit-level detector error models),
 * computed on the host alone, with no device call: for diagnostics and tests.
 * Layout, not arithmetic: the message update of Section II-B is the same for
 * any layout. Every argument is host memory the caller owns.
 *
 * row_ptr, col_idx, M, N: the matrix as in bpsf_load_code, checked the same
 * way (same errors). info[BPSF_SPARSE_INFO_WORDS] receives: [0] the sparse
 * family index, or -1 when the code takes another kernel family (then
 * nothing else is written and the call returns 0); [1] message cells; [2]
 * WMAX, row positions per check; [3] T, threads per workgroup; [4] CPT,
 * checks per thread (internal check i belongs to thread i mod T); [5] DVMAX;
 * [6] cells left above their bank's share in some half-wave group after the
 * column placement; [7] row positions added over all groups; [8] cells moved
 * to a position whose bank another lane of the group reads.
 * Arrays, each may be NULL: roff [M * WMAX] the cell each internal check
 * reads at each position; rw [M] the positions its half-wave reads (at least
 * its weight); bits [N] first cell | weight << 16 of each internal bit; cperm
 * [N] the caller's bit of each internal bit; rperm [M] the caller's check of
 * each internal check. Cells from info[1] on are padding: DVMAX cells read
 * past the last column, then T * CPT pad cells, +inf when a row reads them
 * (thread t's pad for its check slot i is cell info[1] + DVMAX + t CPT + i).
 */
#define BPSF_SPARSE_INFO_WORDS 9
int bpsf_sparse_layout(const int32_t* row_ptr, const int32_t* col_idx, int32_t M, int32_t N, int32_t* info,
                       uint16_t* roff, uint8_t* rw, uint32_t* bits, uint16_t* cperm, uint16_t* rperm);

/* Message of the last failing call on this thread ("" if none). */
const char* bpsf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BPSF_H */
