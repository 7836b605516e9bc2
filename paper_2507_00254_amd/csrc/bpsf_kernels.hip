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
//   * a wave runs D independent decodes ("slots"); the G = 64/D lanes of slot
//     d are contiguous, and lane (d, q) owns checks c = q + G*k (k < IC) and
//     bits v = q + G*k (k < IV) of that slot;
//   * one message per Tanner edge lives in LDS: the v2c value after the bit
//     phase and the c2v value after the check phase (each phase overwrites the
//     edges it owns in place); layout [edge position j][slot d][check c] with
//     stride MS per slot and CI = D*MS per position, so check-phase accesses
//     are consecutive words and bit-phase gathers are mostly consecutive on
//     quasi-cyclic codes;
//   * the syndrome test is incremental: u = H e (one LDS word per check, laid
//     out like the check items, bit 0 used) is toggled only when a hard
//     decision flips, and a slot has converged when u equals its syndrome; a
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

#include "bpsf_internal.h"
#include "bpsf_tiles.h"

namespace bpsf {

// ------------------------------------------------------------------ types --

template <typename Real> struct RT;

template <> struct RT<float> {
  static __device__ __forceinline__ uint32_t sw(float x) { return __float_as_uint(x); }
  // XOR the sign bit of s into v
  static __device__ __forceinline__ float flip(float v, uint32_t s) {
    return __uint_as_float(__float_as_uint(v) ^ (s & 0x80000000u));
  }
  static __device__ __forceinline__ float absr(float x) { return fabsf(x); }
  static __device__ __forceinline__ float minr(float a, float b) { return fminf(a, b); }
  static __device__ __forceinline__ float maxr(float a, float b) { return fmaxf(a, b); }
  static __device__ __forceinline__ float med3(float a, float b, float c) {
    return __builtin_amdgcn_fmed3f(a, b, c);
  }
  static __device__ __forceinline__ float from_double(double x) { return (float)x; }
  // 1 - 2^-i: exact in float for i <= 24 and rounded to 1 beyond, as the
  // double value converted to float would be
  static __device__ __forceinline__ float adaptive_alpha(int i) { return 1.0f - ldexpf(1.0f, -i); }
  // sign bit set exactly when x <= 0 (the hard decision of step 4); x is never -0 or NaN here
  static __device__ __forceinline__ uint32_t nonpos_msb(float x) { return __float_as_uint(x) - 1u; }
  // keeps the compiler from re-associating a select with a later multiply
  static __device__ __forceinline__ void opaque(float& a) { asm volatile("" : "+v"(a)); }
};

template <> struct RT<double> {
  static __device__ __forceinline__ uint32_t sw(double x) {
    return (uint32_t)((unsigned long long)__double_as_longlong(x) >> 32);
  }
  static __device__ __forceinline__ double flip(double v, uint32_t s) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    b ^= (unsigned long long)(s & 0x80000000u) << 32;
    return __longlong_as_double((long long)b);
  }
  static __device__ __forceinline__ double absr(double x) { return fabs(x); }
  static __device__ __forceinline__ double minr(double a, double b) { return fmin(a, b); }
  static __device__ __forceinline__ double maxr(double a, double b) { return fmax(a, b); }
  static __device__ __forceinline__ double med3(double a, double b, double c) {
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
  }
  static __device__ __forceinline__ double from_double(double x) { return x; }
  static __device__ __forceinline__ double adaptive_alpha(int i) { return 1.0 - ldexp(1.0, -i); }
  static __device__ __forceinline__ uint32_t nonpos_msb(double x) {
    return (uint32_t)(((unsigned long long)__double_as_longlong(x) - 1ull) >> 32);
  }
  static __device__ __forceinline__ void opaque(double& a) { asm volatile("" : "+v"(a)); }
};

__device__ __forceinline__ long long bcast0ll(long long x) {
  int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
  int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return ((long long)hi << 32) | (unsigned int)lo;
}

// Butterfly reductions over the G contiguous lanes of a slot. Steps inside a
// row of 16 lanes use DPP lane permutations (no LDS traffic).
template <int G, class Op>
__device__ __forceinline__ uint32_t group_reduce(uint32_t x, Op op)
{
  if constexpr (G >= 2) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));  // lane ^ 1
  if constexpr (G >= 4) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));  // lane ^ 2
  if constexpr (G >= 8) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false)); // mirror in 8
  if constexpr (G >= 16) x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false)); // mirror in 16
  if constexpr (G >= 32) x = op(x, (uint32_t)__shfl_xor((int)x, 16));
  if constexpr (G >= 64) x = op(x, (uint32_t)__shfl_xor((int)x, 32));
  return x;
}

struct OpAdd { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; } };
struct OpMax { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; } };

// --------------------------------------------------------------- kernel --

// UL: every bit has the same channel LLR (uniform priors), held in a scalar.
template <typename Real, int D, int IC, int IV, int W, int DV, bool UL, int MODE, bool TRACE>
__global__ __launch_bounds__(64) void bpsf_kernel(Args a)
{
  using T = TileShape<D, IC, IV, W, DV>;
  using R = RT<Real>;
  constexpr int G = T::G, LG = T::LG, RING = T::RING, PL = T::PL, META = T::META;
  constexpr int KMAX = T::KMAX, MS = T::MS, CI = T::CI, MSB = T::MSB;
  static_assert(IC <= 16, "check items are packed into 16-bit column masks");

  extern __shared__ __align__(16) unsigned char smem[];
  const LdsLayout lay = lds_layout(sizeof(Real), W, CI, CI, a.N, DV, RING, META, KMAX, G);
  Real* msg = reinterpret_cast<Real*>(smem + lay.msg);
  uint32_t* uw = reinterpret_cast<uint32_t*>(smem + lay.resid);
  uint16_t* chk = reinterpret_cast<uint16_t*>(smem + lay.chk);
  int32_t* ring_meta = reinterpret_cast<int32_t*>(smem + lay.ring_meta);
  uint32_t* ring_syn = reinterpret_cast<uint32_t*>(smem + lay.ring_syn);
  uint32_t* ring_tb = reinterpret_cast<uint32_t*>(smem + lay.ring_tv);

  const int lane = threadIdx.x;
  const int d = lane >> LG;          // slot
  const int q = lane & (G - 1);      // lane within the slot
  const int M = a.M, N = a.N;
  const Real* __restrict__ llr = reinterpret_cast<const Real*>(a.llr);
  const Real Lu = R::from_double(a.llr_uniform);   // used when UL
  const bool adaptive = !(a.alpha > 0.0);
  const Real alpha_fixed = R::from_double(adaptive ? 1.0 : a.alpha);

  // ---- per-code tables into LDS ------------------------------------------
  for (int i = lane; i < N * DV; i += 64) chk[i] = a.var_chk[i];
  for (int i = lane; i < CI; i += 64) uw[i] = 0u;

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
        const int c = a.var_chk[v * DV + j];
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
  const int cbase = d * MS + q;      // check items: entry of position 0, item 0

  // message reset: a fresh decode starts from c2v = 0, i.e. v2c = L of the
  // edge's bit. Lane i covers entries c = i + 64 h (h < MSB) of every edge
  // position of a slot; with non-uniform priors it keeps the values to write.
  Real rst_val[UL ? 1 : W][UL ? 1 : MSB];
  if constexpr (!UL) {
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int h = 0; h < MSB; ++h) {
        const int c = lane + 64 * h;
        int v = -1;
        if (c < M) v = a.ell_col[c * W + j];
        rst_val[j][h] = v >= 0 ? llr[v] : (Real)0;
      }
  }

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

  // ---- task source ---------------------------------------------------------
  long long n_tasks;
  unsigned long long* next_ctr;
  if constexpr (MODE == MODE_MAIN) {
    n_tasks = a.shots;
    next_ctr = &a.counters[CNT_MAIN_NEXT];
  } else if constexpr (MODE == MODE_CAND) {
    n_tasks = (long long)__atomic_load_n(&a.counters[CNT_FAILED], __ATOMIC_RELAXED) * a.n_trials;
    next_ctr = &a.counters[CNT_CAND_NEXT];
  } else {
    n_tasks = (long long)__atomic_load_n(&a.counters[CNT_FAILED], __ATOMIC_RELAXED);
    next_ctr = &a.counters[CNT_EMIT_NEXT];
  }
  n_tasks = bcast0ll(n_tasks);
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
      if (lane == 0) base = (long long)atomicAdd(next_ctr, (unsigned long long)a.chunk);
      base = bcast0ll(base);
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
      const uint8_t* s = a.syndromes + t * (long long)M;
#pragma unroll
      for (int k = 0; k < IC; ++k) {
        const int c = q + G * k;
        pf_b[k] = c < M ? (uint32_t)s[c] : 0u;
      }
    } else {
      long long f, ti;
      if constexpr (MODE == MODE_CAND) {
        f = t / a.n_trials;
        ti = t - f * a.n_trials;
      } else {
        f = t;
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
      pf_mask = a.trial_masks[ti];
      pf_ti = (int)ti;
      pf_f = (int)f;   // records never exceed the shots of one call (int32, checked on the host)
    }
  };

  // Write the in-flight inputs into the ring.
  auto commit_prefetch = [&]() {
    if (pend_n == 0) return;
    bool valid = d < pend_n;
    if constexpr (MODE == MODE_EMIT) valid = valid && pf_key != KEY_NONE;
    // compact: rank of my entry among valid entries (count q == 0 lanes below)
    const unsigned long long vb = __ballot(valid && q == 0);
    const int rank = __popcll(vb & ((1ull << (d * G)) - 1ull));
    const int nvalid = __popcll(vb);
    if (valid) {
      const int e = (tail + rank) % RING;
      if constexpr (MODE == MODE_MAIN) {
        uint32_t bits = 0;
#pragma unroll
        for (int k = 0; k < IC; ++k) bits |= (pf_b[k] & 1u) << k;
        ring_syn[e * G + q] = bits;
        if (q == 0) {
          const long long t = pend_base + d;
          ring_meta[e * META + 0] = (int32_t)(t & 0xffffffff);
          ring_meta[e * META + 1] = (int32_t)(t >> 32);
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
    const int e = (head + rank) % RING;
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
    // messages of taken slots: v2c = L (c2v = 0 before the first iteration)
    unsigned long long tb = __ballot(take && q == 0);
    while (tb) {
      const int ld = __ffsll((long long)tb) - 1;
      tb &= tb - 1ull;
      const int sbase = (ld >> LG) * MS + lane;
#pragma unroll
      for (int j = 0; j < W; ++j)
#pragma unroll
        for (int h = 0; h < MSB; ++h)
          if (64 * h + lane < MS) {
            if constexpr (UL) msg[j * CI + sbase + 64 * h] = Lu;
            else msg[j * CI + sbase + 64 * h] = rst_val[j][h];
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

    // ---- check phase: c2v from v2c, Eq. (c2v) ----
    Real alpha = alpha_fixed;
    if (adaptive) alpha = R::adaptive_alpha(iter + 1);
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
          for (int j = 0; j < W; ++j) x[(k + 1) & 1][j] = msg[j * CI + cbase + G * (k + 1)];
        }
        Real m1 = R::minr(R::absr(xc[0]), R::absr(xc[1]));
        Real m2 = R::maxr(R::absr(xc[0]), R::absr(xc[1]));
        uint32_t P = R::sw(xc[0]) ^ R::sw(xc[1]);
#pragma unroll
        for (int j = 2; j < W; ++j) {
          m2 = R::med3(m1, m2, R::absr(xc[j]));
          m1 = R::minr(m1, R::absr(xc[j]));
          P ^= R::sw(xc[j]);
        }
        P ^= synbits << (31 - k);                         // (-1)^{s_c}
        Real s1 = R::flip(alpha * m1, P), s2 = R::flip(alpha * m2, P);
        R::opaque(s1);
        R::opaque(s2);
#pragma unroll
        for (int j = 0; j < W; ++j) {
          // the minimum over the other edges: min2 on the edge holding min1
          const Real o = R::flip(R::absr(xc[j]) == m1 ? s2 : s1, R::sw(xc[j]));
          msg[j * CI + cbase + G * k] = o;
          if constexpr (TRACE) {
            const int c = q + G * k;
            if (d == 0 && active && c < M)
              reinterpret_cast<Real*>(a.trace_c2v)[(long long)iter * M * W + c * W + j] = o;
          }
        }
      }
    }
    __syncthreads();
    commit_prefetch();

    // ---- bit phase: marginal, hard decision, next v2c ----
    uint32_t nhb = 0;
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
      while (f) {
        const int k = __builtin_ctz(f);
        f &= f - 1u;
        const int v = q + (k << LG);
#pragma unroll
        for (int i = 0; i < DV; ++i) atomicXor(&uw[d * MS + chk[v * DV + i]], 1u);
      }
    }
    __syncthreads();

    // ---- syndrome test of every slot: u == s on all its checks ----
    uint32_t un = 0;
#pragma unroll
    for (int k = 0; k < IC; ++k) un |= uw[cbase + G * k] ^ (synbits >> k);
    un &= 1u;
    const unsigned long long ub = __ballot(un != 0u);
    const unsigned long long gm = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const bool conv = ((ub >> (d * G)) & gm) == 0ull;
    if (active) iter += 1;
    const int cap = (MODE == MODE_MAIN) ? a.max_iter : a.cand_max_iter;
    const bool stop_ok = conv && !(a.flags & FLAG_NO_EARLY_STOP);
    const bool fin = active && (stop_ok || iter >= cap);

    if (__ballot(fin) != 0ull) {
      if constexpr (MODE == MODE_MAIN) {
        if (fin) {
          uint8_t* out = a.corrections + shot * (long long)N;
#pragma unroll
          for (int k = 0; k < IV; ++k)
            if ((vmask >> k) & 1u) out[q + G * k] = (uint8_t)((hb >> k) & 1u);
          if (q == 0) {
            a.converged[shot] = (uint8_t)conv;
            a.iterations[shot] = iter;
            st_iters += (unsigned long long)iter;
          }
        }
        const bool need = fin && a.k > 0 && (!conv || (a.flags & FLAG_FORCE_PP));
        if (__ballot(need) != 0ull) {
          // flip counts of my bits; key = count << 16 | (0xffff - v): largest
          // count first, then lowest index
          uint32_t key[IV];
#pragma unroll
          for (int k = 0; k < IV; ++k) {
            uint32_t cn = 0;
#pragma unroll
            for (int b = 0; b < PL; ++b) cn |= ((cnt[b] >> k) & 1u) << b;
            key[k] = ((vmask >> k) & 1u) ? ((cn << 16) | (uint32_t)(0xffff - (q + G * k))) : 0u;
          }
          int f = 0;
          if (need && q == 0) f = (int)atomicAdd(&a.counters[CNT_FAILED], 1ull);
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
          // top(flip_count, |Phi|), one bit per round
          for (int j = 0; j < a.k; ++j) {
            uint32_t best = 0;
#pragma unroll
            for (int k = 0; k < IV; ++k) best = key[k] > best ? key[k] : best;
            best = group_reduce<G>(best, OpMax());
            const int v = best ? 0xffff - (int)(best & 0xffffu) : 0;   // best > 0 while k <= N
            // my share of column v: my checks among its DV checks, and v itself
            uint32_t tw = 0;
#pragma unroll
            for (int i = 0; i < DV; ++i) {
              const int c = chk[v * DV + i];
              if ((c & (G - 1)) == q) tw ^= 1u << (c >> LG);
            }
            if ((v & (G - 1)) == q) tw |= (uint32_t)((v >> LG) + 1) << 16;
            if (need) {
              r[REC_HDR + G + j * G + q] = (int32_t)tw;
              if (q == 0) r[REC_HDR + G + a.k * G + j] = v;
            }
            if ((v & (G - 1)) == q) {
#pragma unroll
              for (int k = 0; k < IV; ++k)
                if (q + G * k == v) key[k] = 0u;
            }
          }
        }
      } else if constexpr (MODE == MODE_CAND) {
        // weight of the undone correction e = e' + t over the slot
        const uint32_t w = group_reduce<G>((uint32_t)__popc((hb ^ tbits) & vmask), OpAdd());
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
          uint8_t* out = a.corrections + shot * (long long)N;
          const uint32_t e = hb ^ tbits;
#pragma unroll
          for (int k = 0; k < IV; ++k)
            if ((vmask >> k) & 1u) out[q + G * k] = (uint8_t)((e >> k) & 1u);
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

__global__ void bpsf_reset_counters(unsigned long long* c)
{
  if (threadIdx.x < CNT_WORDS) c[threadIdx.x] = 0ull;
}

// ------------------------------------------------------------ dispatch --

template <typename Real, int D, int IC, int IV, int W, int DV, bool UL>
static int launch_tile(int mode, bool trace, const Args& a, int grid, void* stream)
{
  using T = TileShape<D, IC, IV, W, DV>;
  const LdsLayout lay = lds_layout(sizeof(Real), W, T::CI, T::CI, a.N, DV, T::RING, T::META, T::KMAX, T::G);
  const size_t sh = lay.total;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (mode == MODE_MAIN && trace)
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_MAIN, true>), dim3(grid), dim3(64), sh, st, a);
  else if (mode == MODE_MAIN)
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_MAIN, false>), dim3(grid), dim3(64), sh, st, a);
  else if (mode == MODE_CAND)
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_CAND, false>), dim3(grid), dim3(64), sh, st, a);
  else
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_EMIT, false>), dim3(grid), dim3(64), sh, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real, int D, int IC, int IV, int W, int DV, bool UL>
static int occupancy_tile(int mode, const Args& a, int* blocks_per_cu)
{
  using T = TileShape<D, IC, IV, W, DV>;
  const LdsLayout lay = lds_layout(sizeof(Real), W, T::CI, T::CI, a.N, DV, T::RING, T::META, T::KMAX, T::G);
  hipError_t e;
  if (mode == MODE_MAIN)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_MAIN, false>, 64, lay.total);
  else if (mode == MODE_CAND)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_CAND, false>, 64, lay.total);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bpsf_kernel<Real, D, IC, IV, W, DV, UL, MODE_EMIT, false>, 64, lay.total);
  return e == hipSuccess ? 0 : -1;
}

template <typename Real, int D, int IC, int IV, int W, int DV>
static int tile_call(int what, bool ul, int mode, bool trace, const Args& a, int grid, void* st, int* out)
{
  if (ul) return what == 0 ? launch_tile<Real, D, IC, IV, W, DV, true>(mode, trace, a, grid, st)
                            : occupancy_tile<Real, D, IC, IV, W, DV, true>(mode, a, out);
  return what == 0 ? launch_tile<Real, D, IC, IV, W, DV, false>(mode, trace, a, grid, st)
                   : occupancy_tile<Real, D, IC, IV, W, DV, false>(mode, a, out);
}

#define BPSF_TILE_CASE(D_, IC_, IV_, W_, DV_)                                                          \
  if (t.D == D_ && t.IC == IC_ && t.IV == IV_ && t.W == W_ && t.DV == DV_) {                           \
    return fp64 ? tile_call<double, D_, IC_, IV_, W_, DV_>(what, ul, mode, trace, a, grid, st, out)    \
                : tile_call<float, D_, IC_, IV_, W_, DV_>(what, ul, mode, trace, a, grid, st, out);    \
  }

int tile_dispatch(int what, const TileDesc& t, bool fp64, bool ul, int mode, bool trace, const Args& a, int grid,
                  void* st, int* out)
{
  BPSF_TILE_LIST(BPSF_TILE_CASE)
  return -2;   // no such tile compiled
}

int reset_counters(unsigned long long* c, void* stream)
{
  hipLaunchKernelGGL(bpsf_reset_counters, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), c);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace bpsf
