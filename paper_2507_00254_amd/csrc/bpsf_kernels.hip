// BP-SF decoding kernels for gfx950 (MI355X).
//
// Method: flooding normalized min-sum BP (paper Section II-B, steps 1-4 and
// Eq. (c2v)) with per-bit oscillation counting, top-|Phi| selection, trial
// syndromes s' = s + t H^T, one short BP per trial and undoing the flip on the
// output (Algorithm 1); among successful trials the lightest undone correction
// is kept (Section IV: Chase-style minimum-weight selection), or the lowest
// successful trial index ("first valid codeword").
//
// Execution model (one wavefront = one workgroup, persistent):
//   * a wave runs D independent decodes ("slots"; D chosen per launch); the
//     G = 64/D lanes of slot d are contiguous, and lane (d, q) owns the block
//     of checks c = q*IC + k (k < IC) and the bits v = q + G*k (k < IV) of
//     that slot, IC and IV being fixed per kernel family;
//   * one message per Tanner edge lives in LDS: the v2c value after the bit
//     phase and the c2v value after the check phase (each phase overwrites the
//     edges it owns in place); layout [edge position j][slot d][check c] with
//     stride MS = G*IC per slot and CI = 64*IC per position. A lane's check
//     items then sit at IC*lane + k whatever D is: compile-time offsets, and
//     with IC odd the 32 lanes of a half-wave hit distinct banks. Bit-phase
//     gathers of consecutive bits are mostly consecutive on quasi-cyclic
//     codes;
//   * the syndrome test is incremental: u = H e (16 LDS bits per lane, bit k
//     for its check item k) is toggled only when a hard decision flips, and
//     a slot has converged when u equals its syndrome; a
//     refilled slot keeps its previous hard decisions as the toggle baseline,
//     so u never needs re-initializing;
//   * flip counts are bit-sliced counters (8 planes) in registers;
//   * a finished slot is refilled at once from an LDS ring of tasks whose
//     inputs were prefetched one iteration earlier (early-exit compaction);
//   * a failed first BP leaves a record holding, per lane, its check bits of
//     s and, for every bit of Phi, the lane's share of that bit's column, so a
//     trial's s' and t are a few XORs away.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bpsf_device.h"
#include "bpsf_internal.h"
#include "bpsf_tiles.h"

namespace bpsf {

// --------------------------------------------------------------- kernel --

// One phase (MODE) of one code: the wave takes the code's tasks until none is
// left and returns once its slots have drained. UL: every bit has the same
// channel LLR (uniform priors), held in a scalar. LAY: layered schedule (the
// checks layer by layer, each reading and updating the bits' posteriors)
// instead of flooding. first, n_first: n_first waves of the launch take
// their first chunk of tasks without the shared counter, this wave chunk
// `first` of them (-1: none), and the counter hands out the chunks after
// those n_first.
// KEEP: the launch may keep trial corrections (Args::trial_bits); without
// it the code that writes and copies them is left out.
template <typename Real, int IC, int IV, int W, int DV, bool UL, int MODE, bool TRACE, bool LAY, bool KEEP>
__device__ __forceinline__ void decode_code(const Args& a, int first, int n_first)
{
  using F = Family<IC, IV, W, DV>;
  using R = RT<Real>;
  constexpr int PL = F::PL, META = F::META, KMAX = F::KMAX, CI = F::CI;
  static_assert(!LAY || W % 2 == 0, "the layered tables are copied as 32-bit words");
  // launch geometry (uniform)
  const int D = a.D;
  const int LG = 6 - __builtin_ctz((unsigned)D);   // log2 of the lanes per slot
  const int G = 1 << LG;
  const int MS = G * IC;                           // message entries per slot and edge position
  const int RING = 2 * D;                          // prefetched tasks (a power of two)

  extern __shared__ __align__(16) unsigned char smem[];
  const LdsLayout lay = lds_layout(sizeof(Real), W, CI, a.M, a.N, DV, D, UL, META, LAY, IV);
  Real* msg = reinterpret_cast<Real*>(smem + lay.msg);
  // u = H e: lane g's 16 bits hold its check items (bit k = item k); XORed
  // as 32-bit words, read as one u16 per lane
  uint32_t* uw = reinterpret_cast<uint32_t*>(smem + lay.resid);
  const uint16_t* uw16 = reinterpret_cast<const uint16_t*>(smem + lay.resid);
  // checks of every bit, as (owner lane within the slot) << 4 | item
  uint16_t* chk = reinterpret_cast<uint16_t*>(smem + lay.chk);
  Real* lrow = reinterpret_cast<Real*>(smem + lay.lrow);
  int32_t* ring_meta = reinterpret_cast<int32_t*>(smem + lay.ring_meta);
  uint16_t* ring_syn = reinterpret_cast<uint16_t*>(smem + lay.ring_syn);
  uint32_t* ring_tb = reinterpret_cast<uint32_t*>(smem + lay.ring_tb);
  Real* lpost = reinterpret_cast<Real*>(smem + lay.lpost);          // LAY: [slot][G*IV] posteriors
  uint16_t* ellw = reinterpret_cast<uint16_t*>(smem + lay.ellw);    // LAY: [M][W] bit of each edge

  const int lane = threadIdx.x;
  const int d = lane >> LG;          // slot
  const int q = lane & (G - 1);      // lane within the slot
  const int M = a.M, N = a.N;
  const Real* __restrict__ llr = reinterpret_cast<const Real*>(a.llr);
  const Real Lu = R::from_double(a.llr_uniform);   // used when UL
  const bool adaptive = !(a.alpha > 0.0);
  const Real alpha_fixed = R::from_double(adaptive ? 1.0 : a.alpha);

  // ---- task source ---------------------------------------------------------
  long long n_tasks;
  unsigned long long* next_ctr;
  if constexpr (MODE == MODE_MAIN) {
    n_tasks = a.task_count ? (long long)__atomic_load_n(a.task_count, __ATOMIC_RELAXED) : a.shots;
    next_ctr = &a.counters[CNT_MAIN_NEXT];
  } else if constexpr (MODE == MODE_CAND) {
    n_tasks = (long long)__atomic_load_n(&a.counters[CNT_FAILED], __ATOMIC_RELAXED) * a.n_trials;
    next_ctr = &a.counters[CNT_CAND_NEXT];
  } else {
    n_tasks = (long long)__atomic_load_n(&a.counters[CNT_FAILED], __ATOMIC_RELAXED);
    next_ctr = &a.counters[CNT_EMIT_NEXT];
  }
  n_tasks = bcast0ll(n_tasks);
  // a wave's own first chunk is tasks [first * chunk, (first + 1) * chunk)
  // and the counter hands out the rest after n_first chunks, so a wave with
  // nothing to do leaves before touching LDS or the counter (small calls
  // launch many such waves)
  first = __builtin_amdgcn_readfirstlane(first);   // wave-uniform
  n_first = __builtin_amdgcn_readfirstlane(n_first);
  if (first >= 0 && (long long)first * a.chunk >= n_tasks) return;
  if (first < 0 && (long long)n_first * a.chunk >= n_tasks) return;
  bool first_chunk = first >= 0;

  // ---- per-code tables into LDS ------------------------------------------
  __syncthreads();   // a previous code's phase may still be reading them
  {
    // as 32-bit words (the device table is padded to a whole word), several
    // loads in flight per lane; check c becomes (c / IC) << 4 | c % IC
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.var_chk);
    uint32_t* dst = reinterpret_cast<uint32_t*>(chk);
    const int nw = (N * DV + 1) >> 1;
    auto own = [](uint32_t c) { return ((c / IC) << 4) | (c % IC); };
#pragma unroll 8
    for (int i = lane; i < nw; i += 64) {
      const uint32_t w = src[i];
      dst[i] = own(w & 0xffffu) | (own(w >> 16) << 16);
    }
  }
  if (lane < 32) uw[lane] = 0u;
  if constexpr (LAY) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ell16);
    uint32_t* dst = reinterpret_cast<uint32_t*>(ellw);
    const int nw = (M * W) >> 1;
#pragma unroll 4
    for (int i = lane; i < nw; i += 64) dst[i] = src[i];
  }
  if constexpr (!UL && !LAY) {
    // channel LLR of the bit on every edge (check c, position j): the value a
    // fresh decode's v2c takes there
    for (int i = lane; i < W * M; i += 64) {
      const int j = i / M, c = i - j * M;
      const int v = a.ell_col[c * W + j];
      lrow[i] = v >= 0 ? llr[v] : (Real)0;
    }
  }

  __syncthreads();   // the tables are in place

  // ---- per-lane constants -------------------------------------------------
  // bit items: channel LLR and the byte offsets of their DV edges
  Real Lv[UL ? 1 : IV];
  uint32_t off[IV][DV];
  uint32_t vmask = 0;
  const uint32_t sink = lay.msg + (uint32_t)sizeof(Real) * (uint32_t)(W * CI + lane);
#pragma unroll
  for (int k = 0; k < IV; ++k) {
    const int v = q + G * k;
    if (v < N) {
      vmask |= 1u << k;
      if constexpr (!UL) Lv[k] = llr[v];
#pragma unroll
      for (int j = 0; j < DV; ++j) {
        const int t = chk[v * DV + j];
        const int c = (t >> 4) * IC + (t & 15);
        const int p = a.var_pos[v * DV + j];
        off[k][j] = lay.msg + (uint32_t)sizeof(Real) * (uint32_t)(p * CI + d * MS + c);
      }
    } else {
      if constexpr (!UL) Lv[k] = (Real)0;
#pragma unroll
      for (int j = 0; j < DV; ++j) off[k][j] = sink;
    }
  }
  if constexpr (UL) Lv[0] = Lu;
  const int cbase = d * MS + q * IC;   // check items: entry of position 0, item 0 (= IC * lane)
  // LAY: layer of every check item, one byte each (0xff past M)
  uint32_t lyw[(IC + 3) / 4];
#pragma unroll
  for (int w = 0; w < (IC + 3) / 4; ++w) lyw[w] = 0xffffffffu;
  if constexpr (LAY) {
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      const int c = q * IC + k;
      if (c < M) lyw[k >> 2] &= ~((uint32_t)(0xffu - a.check_layer[c]) << (8 * (k & 3)));
    }
  }
  __syncthreads();

  // ---- slot state (uniform over the G lanes of a slot) --------------------
  bool active = false;
  int iter = 0;                 // iterations done by the current decode
  uint32_t synbits = 0;         // s (or s') of my check items, bit k
  uint32_t hb = 0;              // hard decisions of my bit items, bit k
  uint32_t prevt = 0;           // hard decisions u was last toggled to
  uint32_t prevc = 0;           // previous hard decisions of this decode (flip counting)
  uint32_t cnt[PL];             // bit-sliced flip counts of my bit items
#pragma unroll
  for (int b = 0; b < PL; ++b) cnt[b] = 0;
  uint32_t tbits = 0;           // trial vector t over my bit items
  long long shot = 0;
  int rec = 0, trial = 0, main_iters = 0;

  unsigned long long st_iters = 0, st_conv = 0, st_err = 0;

  const int rstride = a.rec_stride;

  int head = 0, tail = 0;                 // ring positions (monotonic)
  long long cnext = 0, cend = 0;          // reserved task range
  bool exhausted = false;
  int pend_n = 0;                         // tasks whose inputs are in flight
  long long pend_base = 0;
  // in-flight inputs of pending entry dd = d, held by lane (d, q)
  uint32_t pf_b[IC];                      // MAIN: syndrome bytes of my checks
  uint32_t pf_syn = 0;                    // CAND/EMIT: s bits of my checks
  uint32_t pf_tw[KMAX];                   // CAND/EMIT: my share of every Phi column
  uint32_t pf_mask = 0;
  int pf_shot = 0, pf_miters = 0, pf_f = 0, pf_ti = 0;
  long long pf_shot_main = 0;             // MAIN: the shot of my pending task
  unsigned long long pf_key = KEY_NONE;
#pragma unroll
  for (int k = 0; k < IC; ++k) pf_b[k] = 0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) pf_tw[j] = 0;

  // Reserve up to D tasks and start loading their inputs.
  auto issue_prefetch = [&]() {
    if (exhausted || pend_n != 0 || (tail - head) > D) return;
    if (cnext >= cend) {
      long long base = 0;
      if (first_chunk) {
        base = (long long)first * a.chunk;
        first_chunk = false;
      } else {
        if (lane == 0) base = (long long)atomicAdd(next_ctr, (unsigned long long)a.chunk);
        base = bcast0ll(base);
        if (n_first > 0) base += (long long)n_first * a.chunk;
      }
      if (base >= n_tasks) { exhausted = true; return; }
      cnext = base;
      cend = base + a.chunk < n_tasks ? base + a.chunk : n_tasks;
    }
    const long long left = cend - cnext;
    pend_n = left < D ? (int)left : D;
    pend_base = cnext;
    cnext += pend_n;
    if (d >= pend_n) return;
    const long long t = pend_base + d;
    if constexpr (MODE == MODE_MAIN) {
      pf_shot_main = a.task_shot ? (long long)a.task_shot[t] : a.shot_base + t;
      const uint8_t* s = a.syndromes + pf_shot_main * a.syn_stride;
#pragma unroll
      for (int k = 0; k < IC; ++k) {
        const int c = q * IC + k;
        pf_b[k] = c < M ? (uint32_t)s[c] : 0u;
      }
    } else {
      long long f, ti;
      if constexpr (MODE == MODE_CAND) {
        if (a.flags & FLAG_PRUNE) {
          // trial-major: trial 0 of every failed shot, then trial 1, ...; a
          // shot's later trials are then taken after its earlier ones have
          // run, and skipped once one of them has succeeded
          const long long F = n_tasks / a.n_trials;
          ti = t / F;
          f = t - ti * F;
        } else {
          f = t / a.n_trials;
          ti = t - f * a.n_trials;
        }
      } else {
        f = t;
      }
      if (a.rec_list) f = a.rec_list[f];   // this code's f-th record in the shared pool
      if constexpr (MODE == MODE_EMIT) {
        pf_key = a.keys[f];
        ti = pf_key == KEY_NONE ? 0 : (long long)((pf_key >> KEY_ITER_BITS) & 0xffffffffull);
      }
      const int32_t* r = a.records + f * (long long)rstride;
      pf_syn = (uint32_t)r[REC_HDR + q];
#pragma unroll
      for (int j = 0; j < KMAX; ++j)
        if (j < a.k) pf_tw[j] = (uint32_t)r[REC_HDR + G + j * G + q];
      pf_shot = r[REC_SHOT];
      pf_miters = r[REC_MAIN_ITERS];
      pf_mask = a.trial_masks[(long long)pf_shot * a.mask_stride + ti];
      pf_ti = (int)ti;
      pf_f = (int)f;   // records never exceed the shots of one call (int32, checked on the host)
      if constexpr (MODE == MODE_CAND) {
        // lowest-index selection: a trial after one that already succeeded
        // cannot be selected; skip it (a stale key only skips less)
        if (a.flags & FLAG_PRUNE) {
          const unsigned long long kk = __hip_atomic_load(&a.keys[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (kk != KEY_NONE && (long long)((kk >> KEY_ITER_BITS) & 0xffffffffull) < ti) pf_f = -1;
        }
      }
    }
  };

  // Write the in-flight inputs into the ring.
  auto commit_prefetch = [&]() {
    if (pend_n == 0) return;
    bool valid = d < pend_n;
    if constexpr (MODE == MODE_EMIT) valid = valid && pf_key != KEY_NONE;
    if constexpr (MODE == MODE_EMIT && KEEP) {
      if (valid && a.trial_bits && pf_f < a.trial_bits_recs) {
        // the winner's correction as the trial kernel kept it: written here,
        // the task never enters the ring
        // (G through an opaque copy, as in the finish code: no address of
        // my items is kept across the decode loop)
        int Gc = G;
        asm volatile("" : "+s"(Gc));
        const uint32_t ew = a.trial_bits[((long long)pf_f * a.n_trials + pf_ti) * Gc + q];
        uint8_t* out = a.corrections + (long long)pf_shot * a.corr_stride + q;
#pragma unroll 1
        for (int k = 0; k < IV; ++k)
          if ((vmask >> k) & 1u) out[Gc * k] = (uint8_t)((ew >> k) & 1u);
        if (q == 0) {
          a.converged[pf_shot] = 1;
          a.iterations[pf_shot] = pf_miters + (int)(pf_key & ((1ull << KEY_ITER_BITS) - 1ull));
        }
        valid = false;
      }
    }
    if constexpr (MODE == MODE_CAND) valid = valid && pf_f >= 0;   // skipped by pruning
    // compact: rank of my entry among valid entries (count q == 0 lanes below)
    const unsigned long long vb = __ballot(valid && q == 0);
    const int rank = __popcll(vb & ((1ull << (d * G)) - 1ull));
    const int nvalid = __popcll(vb);
    if (valid) {
      const int e = (tail + rank) & (RING - 1);
      if constexpr (MODE == MODE_MAIN) {
        uint32_t bits = 0;
#pragma unroll
        for (int k = 0; k < IC; ++k) bits |= (pf_b[k] & 1u) << k;
        ring_syn[e * G + q] = bits;
        if (q == 0) {
          ring_meta[e * META + 0] = (int32_t)(pf_shot_main & 0xffffffff);
          ring_meta[e * META + 1] = (int32_t)(pf_shot_main >> 32);
        }
      } else {
        // s' = s + t H^T on my checks, and t on my bits
        uint32_t s2 = pf_syn, tb = 0;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          if (j < a.k && ((pf_mask >> j) & 1u)) {
            s2 ^= pf_tw[j] & 0xffffu;
            const uint32_t vi = pf_tw[j] >> 16;
            if (vi) tb |= 1u << (vi - 1u);
          }
        }
        ring_syn[e * G + q] = s2;
        ring_tb[e * G + q] = tb;
        if (q == 0) {
          ring_meta[e * META + 0] = pf_shot;
          ring_meta[e * META + 2] = pf_f;
          ring_meta[e * META + 3] = pf_ti;
          ring_meta[e * META + 4] = pf_miters;
        }
      }
    }
    tail += nvalid;
    pend_n = 0;
  };

  // Start new decodes in every slot that is idle or just finished.
  auto refill = [&](bool want) {
    const unsigned long long wb = __ballot(want && q == 0);
    if (wb == 0ull) return;
    const int avail = tail - head;
    const int rank = __popcll(wb & ((1ull << (d * G)) - 1ull));
    const bool take = want && rank < avail;
    const int e = (head + rank) & (RING - 1);
    const int nw = __popcll(wb);
    head += nw < avail ? nw : avail;
    if (want) active = false;
    if (take) {
      active = true;
      iter = 0;
      prevc = 0;
#pragma unroll
      for (int b = 0; b < PL; ++b) cnt[b] = 0;
      synbits = ring_syn[e * G + q];
      if constexpr (LAY) {
        // posteriors start at the channel LLR
#pragma unroll
        for (int k = 0; k < IV; ++k) lpost[d * (G * IV) + q + G * k] = Lv[UL ? 0 : k];
      }
      if constexpr (MODE == MODE_MAIN) {
        shot = (long long)(uint32_t)ring_meta[e * META + 0] | ((long long)ring_meta[e * META + 1] << 32);
      } else {
        tbits = ring_tb[e * G + q];
        shot = ring_meta[e * META + 0];
        rec = ring_meta[e * META + 2];
        trial = ring_meta[e * META + 3];
        main_iters = ring_meta[e * META + 4];
      }
    }
    // messages of taken slots: v2c = L (c2v = 0 before the first iteration;
    // LAY keeps c2v, which starts at 0); the whole wave writes one slot at a time
    unsigned long long tb = __ballot(take && q == 0);
    while (tb) {
      const int ld = __ffsll((long long)tb) - 1;
      tb &= tb - 1ull;
      const int sbase = (ld >> LG) * MS;
      for (int c = lane; c < MS; c += 64) {
#pragma unroll
        for (int j = 0; j < W; ++j) {
          if constexpr (LAY) msg[j * CI + sbase + c] = (Real)0;
          else if constexpr (UL) msg[j * CI + sbase + c] = Lu;
          else msg[j * CI + sbase + c] = c < M ? lrow[j * M + c] : (Real)0;
        }
      }
    }
  };

  // ---- prime ----------------------------------------------------------------
  __syncthreads();
  issue_prefetch();
  commit_prefetch();
  __syncthreads();
  refill(true);
  __syncthreads();
  issue_prefetch();

  // ---- main loop ------------------------------------------------------------
  for (;;) {
    const bool any_active = __ballot(active) != 0ull;
    if (!any_active && exhausted && pend_n == 0 && tail == head) break;

    Real alpha = alpha_fixed;
    if (adaptive) alpha = R::adaptive_alpha(iter + 1);
    uint32_t nhb = 0;
    if constexpr (LAY) {
      // ---- layered sweep: per layer, every check of the layer reads the
      // posteriors of its bits less its own last c2v, applies Eq. (c2v) and
      // adds its new c2v back; checks of one layer share no bit ----
      Real* lp = lpost + d * (G * IV);
      for (int L = 0; L < a.n_layers; ++L) {
        uint32_t lm = 0;
#pragma unroll
        for (int k = 0; k < IC; ++k) lm |= (((lyw[k >> 2] >> (8 * (k & 3))) & 0xffu) == (uint32_t)L ? 1u : 0u) << k;
        while (lm) {
          const int k = __builtin_ctz(lm);
          lm &= lm - 1u;
          const int c = q * IC + k;
          Real x[W];
          int vb[W];
#pragma unroll
          for (int j = 0; j < W; ++j) {
            vb[j] = ellw[c * W + j];
            x[j] = lp[vb[j]] - msg[j * CI + cbase + k];
          }
          Real m1 = R::minr(R::absr(x[0]), R::absr(x[1]));
          Real m2 = R::maxr(R::absr(x[0]), R::absr(x[1]));
#pragma unroll
          for (int j = 2; j < W; ++j) {
            m2 = R::med3(m1, m2, R::absr(x[j]));
            m1 = R::minr(m1, R::absr(x[j]));
          }
          // sign parity, (-1)^{s_c} included, in bit 31; two signs per op
          uint32_t P = (synbits >> k) << 31;
#pragma unroll
          for (int j = 0; j + 1 < W; j += 2) P = xor3(P, R::sw(x[j]), R::sw(x[j + 1]));
          if constexpr (W % 2 != 0) P ^= R::sw(x[W - 1]);
          Real s1 = R::flip(alpha * m1, P), s2 = R::flip(alpha * m2, P);
          R::opaque(s1);
          R::opaque(s2);
#pragma unroll
          for (int j = 0; j < W; ++j) {
            const Real o = R::flip(R::absr(x[j]) == m1 ? s2 : s1, R::sw(x[j]));
            msg[j * CI + cbase + k] = o;
            lp[vb[j]] = x[j] + o;
            if constexpr (TRACE) {
              if (d == 0 && active && c < M)
                reinterpret_cast<Real*>(a.trace_c2v)[(long long)iter * M * W + c * W + j] = o;
            }
          }
        }
        __syncthreads();   // the next layer reads these posteriors
      }
      commit_prefetch();
      // hard decisions from the posteriors of my bits
#pragma unroll
      for (int k = IV - 1; k >= 0; --k) {
        const Real lout = lp[q + G * k];
        nhb = __builtin_amdgcn_alignbit(nhb, R::nonpos_msb(lout), 31);
        if constexpr (TRACE) {
          const int v = q + G * k;
          if (d == 0 && active && v < N) reinterpret_cast<Real*>(a.trace_lout)[(long long)iter * N + v] = lout;
        }
      }
    } else {
      // ---- check phase: c2v from v2c, Eq. (c2v) ----
      {
        // loads of item k+1 are issued before the stores of item k
        Real x[2][W];
#pragma unroll
        for (int j = 0; j < W; ++j) x[0][j] = msg[j * CI + cbase];
#pragma unroll
        for (int k = 0; k < IC; ++k) {
          Real (&xc)[W] = x[k & 1];
          if (k + 1 < IC) {
#pragma unroll
            for (int j = 0; j < W; ++j) x[(k + 1) & 1][j] = msg[j * CI + cbase + k + 1];
          }
          Real m1 = R::minr(R::absr(xc[0]), R::absr(xc[1]));
          Real m2 = R::maxr(R::absr(xc[0]), R::absr(xc[1]));
#pragma unroll
          for (int j = 2; j < W; ++j) {
            m2 = R::med3(m1, m2, R::absr(xc[j]));
            m1 = R::minr(m1, R::absr(xc[j]));
          }
          // sign parity, (-1)^{s_c} included, in bit 31; two signs per op
          uint32_t P = synbits << (31 - k);
#pragma unroll
          for (int j = 0; j + 1 < W; j += 2) P = xor3(P, R::sw(xc[j]), R::sw(xc[j + 1]));
          if constexpr (W % 2 != 0) P ^= R::sw(xc[W - 1]);
          Real s1 = R::flip(alpha * m1, P), s2 = R::flip(alpha * m2, P);
          R::opaque(s1);
          R::opaque(s2);
#pragma unroll
          for (int j = 0; j < W; ++j) {
            // the minimum over the other edges: min2 on the edge holding min1
            const Real o = R::flip(R::absr(xc[j]) == m1 ? s2 : s1, R::sw(xc[j]));
            msg[j * CI + cbase + k] = o;
            if constexpr (TRACE) {
              const int c = q * IC + k;
              if (d == 0 && active && c < M)
                reinterpret_cast<Real*>(a.trace_c2v)[(long long)iter * M * W + c * W + j] = o;
            }
          }
        }
      }
      __syncthreads();
      commit_prefetch();

      // ---- bit phase: marginal, hard decision, next v2c ----
      {
        // every gather is issued before the first store of this phase
        Real cv[IV][DV];
#pragma unroll
        for (int k = 0; k < IV; ++k)
#pragma unroll
          for (int j = 0; j < DV; ++j) cv[k][j] = *reinterpret_cast<const Real*>(smem + off[k][j]);
#pragma unroll
        for (int k = IV - 1; k >= 0; --k) {
          // prefix sums in ascending check order starting from the channel LLR
          Real pre[DV + 1];
          pre[0] = Lv[UL ? 0 : k];
#pragma unroll
          for (int j = 0; j < DV; ++j) pre[j + 1] = pre[j] + cv[k][j];
          const Real lout = pre[DV];
#pragma unroll
          for (int j = 0; j < DV; ++j) {
            Real acc = pre[j];
#pragma unroll
            for (int i = j + 1; i < DV; ++i) acc = acc + cv[k][i];
            *reinterpret_cast<Real*>(smem + off[k][j]) = acc;   // v2c for the next iteration
          }
          // shift the hard decision of item k in (items run from IV-1 down to 0)
          nhb = __builtin_amdgcn_alignbit(nhb, R::nonpos_msb(lout), 31);
          if constexpr (TRACE) {
            const int v = q + G * k;
            if (d == 0 && active && v < N) reinterpret_cast<Real*>(a.trace_lout)[(long long)iter * N + v] = lout;
          }
        }
      }
    }
    if (active) hb = nhb & vmask;       // an idle slot keeps its bits, so u stays H e
    if constexpr (MODE == MODE_MAIN) {
      const uint32_t fc = hb ^ prevc;
      prevc = hb;
      uint32_t carry = fc;
#pragma unroll
      for (int b = 0; b < PL; ++b) {
        const uint32_t t = cnt[b] & carry;
        cnt[b] ^= carry;
        carry = t;
      }
    }
    // u follows the hard decisions: toggle the checks of every bit that changed
    {
      uint32_t f = hb ^ prevt;
      prevt = hb;
      int ubase = d * (G >> 1);   // my slot's first word of u
      asm volatile("" : "+v"(ubase));
      while (f) {
        const int k = __builtin_ctz(f);
        f &= f - 1u;
        const int v = q + (k << LG);
        // the bit's checks are all read before the first toggle (a toggle
        // could alias a later read as far as the compiler knows, which would
        // serialize every read behind the previous toggle)
        uint32_t t[DV];
#pragma unroll
        for (int i = 0; i < DV; ++i) t[i] = chk[v * DV + i];
#pragma unroll
        for (int i = 0; i < DV; ++i) atomicXor(&uw[ubase + (t[i] >> 5)], 1u << (t[i] & 31u));
      }
    }
    __syncthreads();

    // ---- syndrome test of every slot: u == s on all its checks ----
    // (the lane index through an opaque copy: its LDS address is not worth a
    // register across the loop)
    int ul = lane;
    asm volatile("" : "+v"(ul));
    const uint32_t un = ((uint32_t)uw16[ul] ^ synbits) & ((1u << IC) - 1u);
    const unsigned long long ub = __ballot(un != 0u);
    const unsigned long long gm = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const bool conv = ((ub >> (d * G)) & gm) == 0ull;
    if (active) iter += 1;
    const int cap = (MODE == MODE_MAIN) ? a.max_iter : a.cand_max_iter;
    const bool stop_ok = conv && !(a.flags & FLAG_NO_EARLY_STOP);
    bool fin = active && (stop_ok || iter >= cap);
    if constexpr (MODE == MODE_CAND) {
      // stop a trial once a lower-index trial of its shot has succeeded
      if ((a.flags & FLAG_PRUNE) && __ballot(active && !fin && (iter & 1) == 0) != 0ull) {
        unsigned long long kk = KEY_NONE;
        if (active && q == 0) kk = __hip_atomic_load(&a.keys[rec], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        kk = __shfl(kk, d * G);
        if (active && (iter & 1) == 0 && kk != KEY_NONE && (int)((kk >> KEY_ITER_BITS) & 0xffffffffull) < trial)
          fin = true;
      }
    }

    if (__ballot(fin) != 0ull) {
      // G through an opaque copy: keeps the compiler from hoisting the bit
      // offsets q + G*k of every item out of the main loop (registers held
      // across the whole decode otherwise)
      int Gf = G;
      asm volatile("" : "+s"(Gf));
      if constexpr (MODE == MODE_MAIN) {
        if (fin) {
          uint8_t* out = a.corrections + shot * a.corr_stride;
#pragma unroll
          for (int k = 0; k < IV; ++k)
            if ((vmask >> k) & 1u) out[q + Gf * k] = (uint8_t)((hb >> k) & 1u);
          if (q == 0) {
            a.converged[shot] = (uint8_t)conv;
            a.iterations[shot] = iter;
            st_iters += (unsigned long long)iter;
          }
        }
        const bool need = fin && a.k > 0 && (!conv || (a.flags & FLAG_FORCE_PP));
        if (__ballot(need) != 0ull) {
          // my bits not yet taken into Phi
          uint32_t avail = vmask;
          int f = 0;
          if (need && q == 0) {
            f = (int)atomicAdd(&a.counters[CNT_FAILED], 1ull);
            if (a.rec_list) {
              const int i = f;
              f = (int)atomicAdd(a.rec_alloc, 1ull);
              a.rec_list[i] = f;
            }
          }
          f = __shfl(f, d * G);
          int32_t* r = a.records + (long long)f * rstride;
          if (need) {
            if (q == 0) {
              r[REC_SHOT] = (int32_t)shot;
              r[REC_MAIN_ITERS] = iter;
              r[REC_MAIN_CONV] = conv ? 1 : 0;
              a.keys[f] = KEY_NONE;
            }
            r[REC_HDR + q] = (int32_t)synbits;
          }
          // top(flip_count, |Phi|), one bit per round: the largest count
          // first, then the lowest index. My candidate comes from the
          // bit-sliced counts, highest plane first (the set of my available
          // bits with the largest count, and that count); its key is
          // count << 16 | (0xffff - v), and the slot's maximum key wins.
          for (int j = 0; j < a.k; ++j) {
            uint32_t cand = avail, cn = 0;
#pragma unroll
            for (int b = PL - 1; b >= 0; --b) {
              const uint32_t c1 = cand & cnt[b];
              cand = c1 ? c1 : cand;
              cn |= c1 ? (1u << b) : 0u;
            }
            uint32_t best = cand ? (cn << 16) | (uint32_t)(0xffff - (q + Gf * __builtin_ctz(cand))) : 0u;
            best = group_reduce(best, G, OpMax());
            const int v = best ? 0xffff - (int)(best & 0xffffu) : 0;   // best > 0 while k <= N
            // my share of column v: my checks among its DV checks, and v itself
            uint32_t tw = 0;
#pragma unroll
            for (int i = 0; i < DV; ++i) {
              const int t = chk[v * DV + i];
              if ((t >> 4) == q) tw ^= 1u << (t & 15);
            }
            if ((v & (G - 1)) == q) tw |= (uint32_t)((v >> LG) + 1) << 16;
            if (need) {
              r[REC_HDR + G + j * G + q] = (int32_t)tw;
              if (q == 0) r[REC_HDR + G + a.k * G + j] = v;
            }
            if ((v & (G - 1)) == q) avail &= ~(1u << (v >> LG));
          }
        }
      } else if constexpr (MODE == MODE_CAND) {
        // weight of the undone correction e = e' + t over the slot
        const uint32_t w = group_reduce((uint32_t)__popc((hb ^ tbits) & vmask), G, OpAdd());
        if constexpr (KEEP) {
          if (fin && conv && a.trial_bits && rec < a.trial_bits_recs)
            a.trial_bits[((long long)rec * a.n_trials + trial) * G + q] = (hb ^ tbits) & vmask;
        }
        if (fin && q == 0) {
          st_iters += (unsigned long long)iter;
          if (conv) {
            st_conv += 1;
            const unsigned long long kw = a.select_first ? 0ull : (unsigned long long)w;
            const unsigned long long key = (kw << KEY_WEIGHT_SHIFT) |
                                           ((unsigned long long)(uint32_t)trial << KEY_ITER_BITS) |
                                           (unsigned long long)iter;
            atomicMin(&a.keys[rec], key);
          }
        }
      } else {  // MODE_EMIT
        if (fin) {
          uint8_t* out = a.corrections + shot * a.corr_stride;
          const uint32_t e = hb ^ tbits;
#pragma unroll
          for (int k = 0; k < IV; ++k)
            if ((vmask >> k) & 1u) out[q + Gf * k] = (uint8_t)((e >> k) & 1u);
          if (q == 0) {
            a.converged[shot] = 1;
            a.iterations[shot] = main_iters + iter;
            st_iters += (unsigned long long)iter;
            if (!conv) st_err += 1;
          }
        }
      }
    }

    refill(fin || !active);
    __syncthreads();
    issue_prefetch();
  }

  // ---- statistics -------------------------------------------------------------
  const int sidx = MODE == MODE_MAIN ? ST_MAIN_ITERS : (MODE == MODE_CAND ? ST_CAND_ITERS : ST_EMIT_ITERS);
  if (st_iters) atomicAdd(&a.counters[sidx], st_iters);
  if (st_conv) atomicAdd(&a.counters[ST_CAND_CONV], st_conv);
  if (st_err) atomicAdd(&a.counters[ST_ERRORS], st_err);
  if (lane == 0) atomicAdd(&a.counters[ST_WAVES], 1ull);
}

// Waves per SIMD the register allocator keeps room for: three for the float
// kernels of the row-weight-6 family with uniform priors, whose LDS allows ten
// waves per CU (a few registers over the limit would cut that to eight); the
// mixed kernel of that family too (nine to ten waves per CU by its LDS)
template <typename Real, int W, bool UL, bool TRACE, bool LAY>
constexpr int min_waves_per_simd() { return (sizeof(Real) == 4 && W == 6 && UL && !TRACE && !LAY) ? 3 : 1; }

template <typename Real, int IC, int IV, int W, int DV, bool UL, int MODE, bool TRACE, bool LAY>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(min_waves_per_simd<Real, W, UL, TRACE, LAY>()))) void bpsf_kernel(Args a)
{
  const int b = (int)blockIdx.x;
  __builtin_assume(b >= 0);
  decode_code<Real, IC, IV, W, DV, UL, MODE, TRACE, LAY, true>(a, b, (int)gridDim.x);
}

// ------------------------------------------------------- mixed launches --

// Tasks of a phase of one code already taken (a lower bound: other waves may
// be taking more).
template <int MODE>
__device__ __forceinline__ long long phase_taken(const Args& a)
{
  const int ctr = MODE == MODE_MAIN ? CNT_MAIN_NEXT : (MODE == MODE_CAND ? CNT_CAND_NEXT : CNT_EMIT_NEXT);
  return (long long)__atomic_load_n(&a.counters[ctr], __ATOMIC_RELAXED);
}

// Tasks of a phase of one code (as decode_code counts them).
template <int MODE>
__device__ __forceinline__ long long phase_tasks(const Args& a)
{
  if constexpr (MODE == MODE_MAIN)
    return a.task_count ? (long long)__atomic_load_n(a.task_count, __ATOMIC_RELAXED) : a.shots;
  const long long f = (long long)__atomic_load_n(&a.counters[CNT_FAILED], __ATOMIC_RELAXED);
  return MODE == MODE_CAND ? f * a.n_trials : f;
}

// One phase over several codes of one family: every wave starts on the code
// under the point (b + 1/2) / grid of the cumulative estimated work and then
// takes the codes after it in turn, so waves whose code runs out help the
// others.
// SMALL (calls of at most 65536 shots): the waves that start on a code take
// their first chunk of its tasks by their rank among those waves, not from
// the code's counter (a small call launches far more waves than it has
// chunks, and every counter atomic of a wave that finds nothing costs the
// others a round trip on the same word), and the trials keep their
// corrections. Larger calls take every chunk from the counters and keep no
// corrections: that form's registers leave their long phases about 2%
// faster.
template <typename Real, int IC, int IV, int W, int DV, bool UL, int MODE, bool SMALL>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(min_waves_per_simd<Real, W, UL, false, false>()))) void bpsf_mixed_kernel(const MixArgs m)
{
  if constexpr (SMALL) {
    // every code's task count in one round trip: lane c loads code c's
    const int lane = threadIdx.x;
    long long tasks = 0;
    if (lane < m.n_codes) tasks = phase_tasks<MODE>(m.code[lane]);
    float w[MIX_MAX_CODES];
    float total = 0.f;
#pragma unroll
    for (int c = 0; c < MIX_MAX_CODES; ++c) {
      const long long tc = ((long long)__builtin_amdgcn_readlane((int)(tasks >> 32), c) << 32) |
                           (unsigned int)__builtin_amdgcn_readlane((int)(tasks & 0xffffffff), c);
      w[c] = c < m.n_codes ? (float)tc * m.cost[c] : 0.f;
      total += w[c];
    }
    // code c (with work) starts the waves whose point lies in [P_c, P_c + w_c),
    // P_c the work of the codes before it: waves [lo_c, lo_c + nw_c)
    auto point = [&](int b) { return ((float)b + 0.5f) / (float)gridDim.x * total; };
    auto first_at = [&](float x) {   // first wave whose point is at or past x
      int lo = 0, hi = (int)gridDim.x;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (point(mid) >= x) hi = mid;
        else lo = mid + 1;
      }
      return lo;
    };
    int lo_w[MIX_MAX_CODES], nw[MIX_MAX_CODES];
    float pc = 0.f;
#pragma unroll
    for (int c = 0; c < MIX_MAX_CODES; ++c) {
      lo_w[c] = w[c] > 0.f ? first_at(pc) : 0;
      pc += w[c];
    }
    int next_lo = (int)gridDim.x;
#pragma unroll
    for (int c = MIX_MAX_CODES - 1; c >= 0; --c) {
      nw[c] = w[c] > 0.f ? next_lo - lo_w[c] : 0;
      if (w[c] > 0.f) next_lo = lo_w[c];
    }
    const int b = (int)blockIdx.x;
    // kept across the codes' decodes in one vector register, lane c holding
    // nw_c (scalar registers are the scarce ones here)
    int c0 = 0, r0 = -1, nw_lane = 0;
#pragma unroll
    for (int c = 0; c < MIX_MAX_CODES; ++c) {
      if (nw[c] > 0 && b >= lo_w[c] && b < lo_w[c] + nw[c]) {
        c0 = c;
        r0 = b - lo_w[c];
      }
      if (lane == c) nw_lane = nw[c];
    }
    for (int i = 0; i < m.n_codes; ++i) {
      const int c = (c0 + i) % m.n_codes;
      const int nf = __builtin_amdgcn_readlane(nw_lane, c);
      if (i > 0) {
        // skip the table set-up of a code whose tasks are all taken: its
        // waves' first chunks and what its counter has handed out (read afresh)
        long long t = 0, nt = 0;
        if (lane == 0) {
          t = phase_taken<MODE>(m.code[c]);
          nt = phase_tasks<MODE>(m.code[c]);
        }
        if (bcast0ll(nt) - bcast0ll(t) - (long long)nf * m.code[c].chunk <= 0) continue;
      }
      decode_code<Real, IC, IV, W, DV, UL, MODE, false, false, true>(m.code[c], i == 0 ? r0 : -1, nf);
    }
  } else {
    // every code's task and taken counts in one round trip: lane c loads code c's
    const int lane = threadIdx.x;
    long long tasks = 0, taken = 0;
    if (lane < m.n_codes) {
      tasks = phase_tasks<MODE>(m.code[lane]);
      taken = phase_taken<MODE>(m.code[lane]);
    }
    float w[MIX_MAX_CODES];
    long long ntask[MIX_MAX_CODES], left[MIX_MAX_CODES];
    float total = 0.f;
#pragma unroll
    for (int c = 0; c < MIX_MAX_CODES; ++c) {
      const long long tc = ((long long)__builtin_amdgcn_readlane((int)(tasks >> 32), c) << 32) |
                           (unsigned int)__builtin_amdgcn_readlane((int)(tasks & 0xffffffff), c);
      const long long tk = ((long long)__builtin_amdgcn_readlane((int)(taken >> 32), c) << 32) |
                           (unsigned int)__builtin_amdgcn_readlane((int)(taken & 0xffffffff), c);
      w[c] = c < m.n_codes ? (float)tc * m.cost[c] : 0.f;
      ntask[c] = tc;
      left[c] = c < m.n_codes ? tc - tk : 0;
      total += w[c];
    }
    const float at = ((float)blockIdx.x + 0.5f) / (float)gridDim.x * total;
    int c0 = 0;
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < MIX_MAX_CODES; ++c) {
      if (acc > at || w[c] <= 0.f) continue;
      c0 = c;
      acc += w[c];
    }
    for (int i = 0; i < m.n_codes; ++i) {
      const int c = (c0 + i) % m.n_codes;
      // skip the table set-up of a code whose tasks are all taken (counts read
      // afresh for every code after the first)
      long long rem = 0, nt = 0;
#pragma unroll
      for (int cc = 0; cc < MIX_MAX_CODES; ++cc)
        if (cc == c) {
          rem = left[cc];
          nt = ntask[cc];
        }
      if (i > 0 && rem > 0) {
        long long t = 0;
        if (lane == 0) t = phase_taken<MODE>(m.code[c]);
        rem = nt - bcast0ll(t);
      }
      if (rem <= 0) continue;
      decode_code<Real, IC, IV, W, DV, UL, MODE, false, false, false>(m.code[c], -1, 0);
    }
  }
}

// Each block takes a contiguous slice of the shots: it counts the slice's
// shots of every code in LDS, reserves each code's range of the lists with
// one global atomic, then places the shots (one LDS atomic per wave and code
// in both passes). Order inside a code's list is arbitrary; results do not
// depend on it.
__global__ __launch_bounds__(256) void bpsf_bucket_kernel(BucketArgs b)
{
  __shared__ unsigned int cnt[MIX_MAX_CODES];
  __shared__ unsigned long long base[MIX_MAX_CODES];
  const int tid = threadIdx.x, lane = tid & 63;
  const long long per = (b.shots + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = lo + per < b.shots ? lo + per : b.shots;
  if (tid < MIX_MAX_CODES) cnt[tid] = 0u;
  __syncthreads();
  for (long long i0 = lo; i0 < hi; i0 += blockDim.x) {
    const long long i = i0 + tid;
    int c = -1;
    if (i < hi) {
      c = b.shot_code[i];
      if (c < 0 || c >= b.n_codes) {
        atomicAdd(b.bad, 1ull);
        c = -1;
      }
    }
    for (int cc = 0; cc < b.n_codes; ++cc) {
      const unsigned long long mine = __ballot(c == cc);
      if (mine != 0ull && lane == __ffsll((long long)mine) - 1) atomicAdd(&cnt[cc], (unsigned)__popcll(mine));
    }
  }
  __syncthreads();
  if (tid < b.n_codes) {
    base[tid] = cnt[tid] ? atomicAdd(b.counts[tid], (unsigned long long)cnt[tid]) : 0ull;
    cnt[tid] = 0u;
  }
  __syncthreads();
  for (long long i0 = lo; i0 < hi; i0 += blockDim.x) {
    const long long i = i0 + tid;
    int c = -1;
    if (i < hi) {
      c = b.shot_code[i];
      if (c < 0 || c >= b.n_codes) c = -1;
    }
    for (int cc = 0; cc < b.n_codes; ++cc) {
      const unsigned long long mine = __ballot(c == cc);
      if (mine == 0ull) continue;
      const int leader = __ffsll((long long)mine) - 1;
      unsigned int first = 0;
      if (lane == leader) first = atomicAdd(&cnt[cc], (unsigned)__popcll(mine));
      first = __shfl(first, leader);
      if (c == cc) {
        const unsigned int rank = (unsigned)__popcll(mine & ((1ull << lane) - 1ull));
        b.lists[(long long)cc * b.shots + (long long)(base[cc] + first + rank)] = (int32_t)i;
      }
    }
  }
}

__global__ void bpsf_reset_counters(unsigned long long* c, int n)
{
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0ull;
}

// ------------------------------------------------------------ dispatch --

template <typename Real, int IC, int IV, int W, int DV, bool UL, int MODE, bool TRACE, bool LAY>
static int run_kernel(int what, const Args& a, size_t lds, int grid, hipStream_t st, int* out)
{
  if (what == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_kernel<Real, IC, IV, W, DV, UL, MODE, TRACE, LAY>,
                                                        64, lds) == hipSuccess ? 0 : -1;
  hipLaunchKernelGGL((bpsf_kernel<Real, IC, IV, W, DV, UL, MODE, TRACE, LAY>), dim3(grid), dim3(64), lds, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real, int IC, int IV, int W, int DV, bool UL, bool LAY>
static int run_sched(int what, int mode, bool trace, const Args& a, size_t lds, int grid, hipStream_t st, int* out)
{
  if (mode == MODE_MAIN)
    return trace ? run_kernel<Real, IC, IV, W, DV, UL, MODE_MAIN, true, LAY>(what, a, lds, grid, st, out)
                 : run_kernel<Real, IC, IV, W, DV, UL, MODE_MAIN, false, LAY>(what, a, lds, grid, st, out);
  if (mode == MODE_CAND)
    return run_kernel<Real, IC, IV, W, DV, UL, MODE_CAND, false, LAY>(what, a, lds, grid, st, out);
  return run_kernel<Real, IC, IV, W, DV, UL, MODE_EMIT, false, LAY>(what, a, lds, grid, st, out);
}

template <typename Real, int IC, int IV, int W, int DV, bool UL>
static int run_mode(int what, int mode, bool trace, bool layered, const Args& a, size_t lds, int grid, hipStream_t st,
                    int* out)
{
  return layered ? run_sched<Real, IC, IV, W, DV, UL, true>(what, mode, trace, a, lds, grid, st, out)
                 : run_sched<Real, IC, IV, W, DV, UL, false>(what, mode, trace, a, lds, grid, st, out);
}

template <typename Real, int IC, int IV, int W, int DV, bool UL, bool SMALL>
static int run_mixed_form(int what, int mode, const MixArgs& m, size_t lds, int grid, hipStream_t st, int* out)
{
  if (what == 1) {
    hipError_t e;
    if (mode == MODE_MAIN)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_mixed_kernel<Real, IC, IV, W, DV, UL, MODE_MAIN, SMALL>, 64, lds);
    else if (mode == MODE_CAND)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_mixed_kernel<Real, IC, IV, W, DV, UL, MODE_CAND, SMALL>, 64, lds);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_mixed_kernel<Real, IC, IV, W, DV, UL, MODE_EMIT, SMALL>, 64, lds);
    return e == hipSuccess ? 0 : -1;
  }
  if (mode == MODE_MAIN)
    hipLaunchKernelGGL((bpsf_mixed_kernel<Real, IC, IV, W, DV, UL, MODE_MAIN, SMALL>), dim3(grid), dim3(64), lds, st, m);
  else if (mode == MODE_CAND)
    hipLaunchKernelGGL((bpsf_mixed_kernel<Real, IC, IV, W, DV, UL, MODE_CAND, SMALL>), dim3(grid), dim3(64), lds, st, m);
  else
    hipLaunchKernelGGL((bpsf_mixed_kernel<Real, IC, IV, W, DV, UL, MODE_EMIT, SMALL>), dim3(grid), dim3(64), lds, st, m);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real, int IC, int IV, int W, int DV, bool UL>
static int run_mixed(int what, bool small, int mode, const MixArgs& m, size_t lds, int grid, hipStream_t st, int* out)
{
  return small ? run_mixed_form<Real, IC, IV, W, DV, UL, true>(what, mode, m, lds, grid, st, out)
               : run_mixed_form<Real, IC, IV, W, DV, UL, false>(what, mode, m, lds, grid, st, out);
}

int family_count()
{
  int n = 0;
#define BPSF_FAMILY_COUNT(IC_, IV_, W_, DV_) ++n;
  BPSF_FAMILY_LIST(BPSF_FAMILY_COUNT)
#undef BPSF_FAMILY_COUNT
  return n;
}

FamilyDesc family_desc(int fam)
{
  int i = 0;
#define BPSF_FAMILY_DESC(IC_, IV_, W_, DV_) \
  if (i++ == fam) return FamilyDesc{IC_, IV_, W_, DV_};
  BPSF_FAMILY_LIST(BPSF_FAMILY_DESC)
#undef BPSF_FAMILY_DESC
  return FamilyDesc{0, 0, 0, 0};
}

int tile_dispatch(int what, const TileDesc& t, bool fp64, bool ul, int mode, bool trace, const Args& a, size_t lds,
                  int grid, void* stream, int* out, bool layered)
{
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int i = 0;
#define BPSF_FAMILY_CASE(IC_, IV_, W_, DV_)                                                                    \
  if (i++ == t.fam) {                                                                                          \
    if (fp64)                                                                                                  \
      return ul ? run_mode<double, IC_, IV_, W_, DV_, true>(what, mode, trace, layered, a, lds, grid, st, out)   \
                : run_mode<double, IC_, IV_, W_, DV_, false>(what, mode, trace, layered, a, lds, grid, st, out); \
    return ul ? run_mode<float, IC_, IV_, W_, DV_, true>(what, mode, trace, layered, a, lds, grid, st, out)      \
              : run_mode<float, IC_, IV_, W_, DV_, false>(what, mode, trace, layered, a, lds, grid, st, out);    \
  }
  BPSF_FAMILY_LIST(BPSF_FAMILY_CASE)
#undef BPSF_FAMILY_CASE
  return -2;   // no such family compiled
}

int mixed_dispatch(int what, int fam, bool fp64, bool ul, bool small, int mode, const MixArgs& m, size_t lds,
                   int grid, void* stream, int* out)
{
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int i = 0;
#define BPSF_FAMILY_MIX(IC_, IV_, W_, DV_)                                                        \
  if (i++ == fam) {                                                                               \
    if (fp64) return ul ? run_mixed<double, IC_, IV_, W_, DV_, true>(what, small, mode, m, lds, grid, st, out) \
                        : run_mixed<double, IC_, IV_, W_, DV_, false>(what, small, mode, m, lds, grid, st, out); \
    return ul ? run_mixed<float, IC_, IV_, W_, DV_, true>(what, small, mode, m, lds, grid, st, out)            \
              : run_mixed<float, IC_, IV_, W_, DV_, false>(what, small, mode, m, lds, grid, st, out);          \
  }
  BPSF_FAMILY_LIST(BPSF_FAMILY_MIX)
#undef BPSF_FAMILY_MIX
  return -2;
}

int bucket_launch(const BucketArgs& b, void* stream)
{
  if (b.shots <= 0) return 0;
  // slices of at least 8192 shots, at most 2048 blocks
  long long blocks = (b.shots + 8191) / 8192;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(bpsf_bucket_kernel, dim3((unsigned)blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), b);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int reset_counters(unsigned long long* c, int n, void* stream)
{
  hipLaunchKernelGGL(bpsf_reset_counters, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), c, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bpsf
