// Internal definitions shared by the BP-SF device kernels and the host runtime.
// Not part of the public ABI (that is include/bpsf.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/bpsf.h"

namespace bpsf {

// Decode phases of one bpsf_decode call, each a persistent launch:
//   MAIN  - BP with oscillation counting on every shot (Algorithm 1, first BP);
//           shots that fail get a record with Phi = top(flip_count, k);
//   CAND  - one short BP per (failed shot, trial vector) on s' = s + t H^T; a
//           successful trial posts its key (weight, trial index, iterations);
//   EMIT  - re-runs each failed shot's winning trial and writes its undone
//           correction (the run is deterministic, so it reproduces the winner).
enum Mode : int { MODE_MAIN = 0, MODE_CAND = 1, MODE_EMIT = 2 };

// Record layout for a shot whose first BP failed (int32 words).
enum : int { REC_SHOT = 0, REC_MAIN_ITERS = 1, REC_MAIN_CONV = 2, REC_HDR = 4 };

// Counters and statistics (uint64 words in the scratch block).
enum : int {
  CNT_MAIN_NEXT = 0,    // next shot to take in MAIN
  CNT_FAILED = 1,       // records written by MAIN
  CNT_CAND_NEXT = 2,    // next (record, trial) task in CAND
  CNT_EMIT_NEXT = 3,    // next record in EMIT
  ST_MAIN_ITERS = 4,    // sum of first-BP iterations
  ST_CAND_ITERS = 5,    // sum of trial-BP iterations
  ST_EMIT_ITERS = 6,    // sum of re-run iterations
  ST_CAND_CONV = 7,     // trials that converged
  ST_ERRORS = 8,        // a re-run that did not reproduce its winner (must stay 0)
  ST_WAVES = 9,         // waves that ran to completion
  CNT_WORDS = 16
};

static constexpr uint64_t KEY_NONE = ~0ull;
static constexpr int KEY_ITER_BITS = 12;     // trial iterations (< 4096)
static constexpr int KEY_TRIAL_BITS = 32;    // trial index
static constexpr int KEY_WEIGHT_SHIFT = KEY_ITER_BITS + KEY_TRIAL_BITS;

struct Args {
  // code (device, immutable)
  int M, N;               // checks, bits
  const uint16_t* var_chk;   // [N][DV] checks of each bit, ascending
  const uint8_t* var_pos;    // [N][DV] position of the bit inside each check's row
  const int32_t* ell_col;    // [M][W] bits of each check, row order (ELL, -1 padded)
  const void* llr;           // [N] channel LLR (float or double)
  const uint8_t* row_w;      // [M] row weights (wide kernels)
  const void* edge_init;     // [W][MP] initial v2c per edge position and padded check (wide kernels)
  const uint8_t* check_layer;   // [M] layer of every check (layered schedule)
  const uint16_t* ell16;        // [M][W] bit of every (check, position) (layered schedule)
  int n_layers;
  // sparse family: checks and bits renumbered by weight ("internal"), edges
  // in column-major order of the internal bits
  int E;                        // edges
  const uint16_t* sp_roff;      // [M][WMAX] edge of every row position, the +inf cell past the weight
  const uint8_t* sp_rw;         // [M] row weights
  const uint32_t* sp_bits;      // [N] first edge of the bit | weight << 16
  const uint16_t* sp_echk;      // [E] internal check of every edge
  const uint16_t* sp_rperm;     // [M] internal check -> caller's check
  const uint16_t* sp_cperm;     // [N] internal bit -> caller's bit
  const uint16_t* sp_cinv;      // [N] caller's bit -> internal bit
  double llr_uniform;        // the common channel LLR when every prior is equal
  // problem (device)
  const uint8_t* syndromes;  // [shots][syn_stride]; the first M bytes of a row are s
  int64_t syn_stride;
  int64_t shots;             // first-BP tasks when task_count is NULL
  uint8_t* corrections;      // [shots][corr_stride]; the first N bytes of a row are written
  int64_t corr_stride;
  uint8_t* converged;        // [shots]
  int32_t* iterations;       // [shots]
  // task mapping of a launch that mixes codes (all NULL for a single code):
  int64_t shot_base;         // first-BP task t -> shot shot_base + t when task_shot is NULL
  const int32_t* task_shot;  // first-BP task t -> shot
  const unsigned long long* task_count;   // number of first-BP tasks of this code
  int32_t* rec_list;         // i-th record of this code -> record index in the shared pool
  unsigned long long* rec_alloc;          // allocation counter of the shared record pool
  int D;                     // decodes per wave of this launch (1, 2, 4, 8 or 16)
  // parameters
  int max_iter, cand_max_iter, k, n_trials, select_first, flags;
  double alpha;              // > 0 fixed; 0 adaptive 1 - 2^-i
  const uint32_t* trial_masks;  // shot i's trial t at [i * mask_stride + t]
  int64_t mask_stride;          // 0: one list for every shot
  // scratch (device)
  int32_t* records;          // [cap][rec_stride] (shared by the codes of a mixed launch)
  int rec_stride;
  int64_t rec_cap;
  unsigned long long* keys;  // [cap]
  unsigned long long* counters;  // [CNT_WORDS] of this code
  // single-code calls: [record][trial][lanes of a decode] words, each lane's
  // bits of every converged trial's undone correction (its own bit items or
  // slots), for the first trial_bits_recs records; the re-run phase copies
  // the winner's for those records instead of decoding it again (NULL:
  // every winner is decoded; mixed calls and the wide family)
  uint32_t* trial_bits;
  int64_t trial_bits_recs;
  // per-iteration records of slot 0 (debug entry point only)
  void* trace_lout;          // [max_iter][N] Real
  void* trace_c2v;           // [max_iter][M*W] Real (row-major edge order)
  int chunk;                 // tasks reserved per counter update
};

enum : int { FLAG_NO_EARLY_STOP = 1, FLAG_FORCE_PP = 2, FLAG_PRUNE = 4, FLAG_LAYERED = 8 };

// Sets the calling thread's message for bpsf_last_error and returns code.
int report_error(int code, const char* msg);

// For the request loop: the device bytes of the scratch of a grouped mixed
// call of up to `shots` shots, and such a call with its scratch in a region
// the caller owns (bpsf_mix_decode_grouped otherwise).
int mix_scratch_bytes(bpsf_mix m, int64_t shots, const bpsf_params* p, size_t* out);
// the same in two steps: the record words per shot that cover every call
// size of the mix (computed once), then the bytes for a call of `shots`
int mix_scratch_stride(bpsf_mix m, const bpsf_params* p, int* out);
size_t mix_scratch_size(int n_codes, int64_t shots, int stride);
// bpsf_decode with its scratch in a region the caller owns (a region sized by
// mix_scratch_bytes for a mix holding the code is large enough)
int decode_in(bpsf_code c, const uint8_t* syndromes, const double* priors, int64_t shots, const bpsf_params* p,
              uint8_t* corrections, uint8_t* converged, int32_t* iterations, void* stream, void* scratch,
              size_t scratch_bytes);
int mix_decode_grouped_in(bpsf_mix m, const int64_t* counts, const uint8_t* syndromes, int64_t syn_stride,
                          const double* const* priors, const bpsf_params* p, uint8_t* corrections,
                          int64_t corr_stride, uint8_t* converged, int32_t* iterations, void* stream,
                          void* scratch, size_t scratch_bytes);

// One launch over several codes: every wave starts on a code chosen in
// proportion to the codes' estimated work and moves on to the next code when
// that code's tasks are taken.
constexpr int MIX_MAX_CODES = 8;
struct MixArgs {
  int n_codes;
  float cost[MIX_MAX_CODES];   // relative cost of one task of the code
  Args code[MIX_MAX_CODES];
};

// Prepass of a mixed launch: shots grouped by code into per-code task lists.
struct BucketArgs {
  const int32_t* shot_code;    // [shots] index of each shot's code
  int64_t shots;
  int n_codes;
  int32_t* lists;              // [n_codes][shots]
  unsigned long long* counts[MIX_MAX_CODES];   // per code: number of listed shots
  unsigned long long* bad;     // shots whose code index is out of range
};

}  // namespace bpsf
