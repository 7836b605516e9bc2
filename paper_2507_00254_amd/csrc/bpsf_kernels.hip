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
//   * the syndrome test is incremental: a residual bitmap r = s + H e (one bit
//     per check, laid out like the check items) is toggled only when a hard
//     decision flips; a slot has converged when its residual bits are zero;
//   * flip counts are bit-sliced counters (8 planes) in registers;
//   * a finished slot is refilled at once from an LDS ring of tasks whose
//     inputs were prefetched one iteration earlier (early-exit compaction).
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
  static __device__ __forceinline__ void opaque(double& a) { asm volatile("" : "+v"(a)); }
};

__device__ __forceinline__ int bcast0(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long bcast0ll(long long x) {
  int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
  int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return ((long long)hi << 32) | (unsigned int)lo;
}

// --------------------------------------------------------------- kernel --

template <typename Real, int D, int IC, int IV, int W, int DV, int MODE, bool TRACE>
__global__ __launch_bounds__(64) void bpsf_kernel(Args a)
{
  using T = TileShape<D, IC, IV, W, DV>;
  using R = RT<Real>;
  constexpr int G = T::G, LG = T::LG, RING = T::RING, PL = T::PL, META = T::META, KG = T::KG;
  constexpr int KMAX = T::KMAX;
  constexpr int NRESET = reset_slots<T>();   // the host keeps MS < G*IC + 32

  extern __shared__ __align__(16) unsigned char smem[];
  const LdsLayout lay = lds_layout(sizeof(Real), W, a.CI, T::RW, a.N, DV, RING, META, KMAX, G);
  Real* msg = reinterpret_cast<Real*>(smem + lay.msg);
  uint32_t* resid = reinterpret_cast<uint32_t*>(smem + lay.resid);
  uint16_t* chk = reinterpret_cast<uint16_t*>(smem + lay.chk);
  int32_t* ring_meta = reinterpret_cast<int32_t*>(smem + lay.ring_meta);
  int32_t* ring_tv = reinterpret_cast<int32_t*>(smem + lay.ring_tv);
  uint32_t* ring_syn = reinterpret_cast<uint32_t*>(smem + lay.ring_syn);

  const int lane = threadIdx.x;
  const int d = lane >> LG;          // slot
  const int q = lane & (G - 1);      // lane within the slot
  const int M = a.M, N = a.N, MS = a.MS, CI = a.CI;
  const Real* __restrict__ llr = reinterpret_cast<const Real*>(a.llr);

  // ---- per-code tables into LDS ------------------------------------------
  for (int i = lane; i < N * DV; i += 64) chk[i] = a.var_chk[i];
  for (int i = lane; i < T::RW; i += 64) resid[i] = 0u;

  // ---- per-lane constants -------------------------------------------------
  // bit items: channel LLR and the byte offsets of their DV edges
  Real Lv[IV];
  uint32_t off[IV][DV];
  uint32_t vmask = 0;
  const uint32_t sink = lay.msg + (uint32_t)sizeof(Real) * (uint32_t)(W * CI + lane);
#pragma unroll
  for (int k = 0; k < IV; ++k) {
    const int v = q + G * k;
    if (v < N) {
      vmask |= 1u << k;
      Lv[k] = llr[v];
#pragma unroll
      for (int j = 0; j < DV; ++j) {
        const int c = a.var_chk[v * DV + j];
        const int p = a.var_pos[v * DV + j];
        off[k][j] = lay.msg + (uint32_t)sizeof(Real) * (uint32_t)(p * CI + d * MS + c);
      }
    } else {
      Lv[k] = (Real)0;
#pragma unroll
      for (int j = 0; j < DV; ++j) off[k][j] = sink;
    }
  }
  // check items: word offsets of position 0 (positions are CI apart)
  const int cbase = d * MS + q;
  // valid check items (c < M)
  uint32_t cmask = 0;
#pragma unroll
  for (int k = 0; k < IC; ++k)
    if (q + G * k < M) cmask |= 1u << k;

  // message reset: a fresh decode starts from c2v = 0, i.e. v2c = L of the
  // edge's bit; every lane covers entries i = lane + 64 r of the slot's
  // W x MS block (r < NR), stored with the value to write
  const int NR = (W * MS + 63) / 64;
  uint32_t rst_off[NRESET];
  Real rst_val[NRESET];
#pragma unroll
  for (int r = 0; r < NRESET; ++r) {
    const int i = lane + 64 * r;
    rst_off[r] = 0xffffffffu;
    rst_val[r] = (Real)0;
    if (r < NR && i < W * MS) {
      const int j = i / MS, c = i - j * MS;
      rst_off[r] = lay.msg + (uint32_t)sizeof(Real) * (uint32_t)(j * CI + c);
      if (c < M) {
        const int v = a.ell_col[c * W + j];
        rst_val[r] = v >= 0 ? llr[v] : (Real)0;
      }
    }
  }

  // ---- slot state (uniform over the G lanes of a slot) --------------------
  bool active = false;
  int iter = 0;                 // iterations done by the current decode
  uint32_t synbits = 0;         // s (or s') of my check items, bit k
  uint32_t hb = 0, prevhb = 0;  // hard decisions of my bit items, bit k
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

  int head = 0, tail = 0;                 // ring positions (monotonic)
  long long cnext = 0, cend = 0;          // reserved task range
  bool exhausted = false;
  int pend_n = 0;                         // tasks whose inputs are in flight
  long long pend_base = 0;
  // in-flight inputs of entry dd = d (lane (dd, q))
  uint32_t pf_b[IC];
  uint32_t pf_syn = 0;
  int pf_shot = 0, pf_miters = 0, pf_f = 0, pf_ti = 0, pf_phi[KG];
  uint32_t pf_mask = 0;
  unsigned long long pf_key = KEY_NONE;
#pragma unroll
  for (int k = 0; k < IC; ++k) pf_b[k] = 0;
#pragma unroll
  for (int r = 0; r < KG; ++r) pf_phi[r] = -1;

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
      const int32_t* r = a.records + f * (long long)a.rec_stride;
      pf_syn = (uint32_t)r[REC_HDR + KMAX + q];
      pf_shot = r[REC_SHOT];
      pf_miters = r[REC_MAIN_ITERS];
#pragma unroll
      for (int rr = 0; rr < KG; ++rr) {
        const int j = q + G * rr;
        pf_phi[rr] = j < a.k ? r[REC_HDR + j] : -1;
      }
      pf_mask = a.trial_masks[ti];
      pf_ti = (int)ti;
      pf_f = (int)f;   // records never exceed the shots of one call (int32 range, checked on the host)
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
        ring_syn[e * G + q] = pf_syn;
#pragma unroll
        for (int rr = 0; rr < KG; ++rr) {
          const int j = q + G * rr;
          if (j < KMAX) ring_tv[e * KMAX + j] = (j < a.k && ((pf_mask >> j) & 1u)) ? pf_phi[rr] : -1;
        }
        if (q == 0) {
          ring_meta[e * META + 0] = pf_shot;
          ring_meta[e * META + 1] = 0;
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
    const int ntake = __popcll(wb) < avail ? __popcll(wb) : avail;
    head += ntake;
    if (want) active = false;
    if (take) {
      active = true;
      iter = 0;
      hb = 0;
      prevhb = 0;
#pragma unroll
      for (int b = 0; b < PL; ++b) cnt[b] = 0;
      synbits = ring_syn[e * G + q];
      if constexpr (MODE == MODE_MAIN) {
        shot = (long long)(uint32_t)ring_meta[e * META + 0] | ((long long)ring_meta[e * META + 1] << 32);
      } else {
        shot = ring_meta[e * META + 0];
        rec = ring_meta[e * META + 2];
        trial = ring_meta[e * META + 3];
        main_iters = ring_meta[e * META + 4];
        tbits = 0;
        for (int j = 0; j < a.k; ++j) {
          const int v = ring_tv[e * KMAX + j];
          if (v >= 0 && (v & (G - 1)) == q) tbits |= 1u << (v >> LG);
        }
      }
    }
    // residual of a taken slot starts at its syndrome: set my bits
    const uint32_t mybit = 1u << (lane & 31);
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      uint32_t* w = &resid[k * 2 + (lane >> 5)];
      if (take) {
        if ((synbits >> k) & 1u) atomicOr(w, mybit);
        else atomicAnd(w, ~mybit);
      }
    }
    // messages of taken slots: v2c = L (c2v = 0 before the first iteration)
    unsigned long long tb = __ballot(take && q == 0);
    while (tb) {
      const int ld = __ffsll((long long)tb) - 1;
      tb &= tb - 1ull;
      const int sd = ld >> LG;
      const uint32_t sofs = (uint32_t)sizeof(Real) * (uint32_t)(sd * MS);
#pragma unroll
      for (int r = 0; r < NRESET; ++r)
        if (rst_off[r] != 0xffffffffu)
          *reinterpret_cast<Real*>(smem + rst_off[r] + sofs) = rst_val[r];
    }
    if constexpr (MODE != MODE_MAIN) {
      __syncthreads();
      // s' = s + t H^T: toggle the checks of every bit in t
      if (take) {
        for (int j = q; j < a.k; j += G) {
          const int v = ring_tv[e * KMAX + j];
          if (v >= 0) {
#pragma unroll
            for (int i = 0; i < DV; ++i) {
              const int c = chk[v * DV + i];
              const int ol = (d << LG) | (c & (G - 1));
              atomicXor(&resid[(c >> LG) * 2 + (ol >> 5)], 1u << (ol & 31));
            }
          }
        }
      }
      __syncthreads();
      if (take) {
        uint32_t s2 = 0;
#pragma unroll
        for (int k = 0; k < IC; ++k) s2 |= ((resid[k * 2 + (lane >> 5)] >> (lane & 31)) & 1u) << k;
        synbits = s2;
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
    Real alpha;
    if (a.alpha > 0.0) alpha = R::from_double(a.alpha);
    else alpha = R::from_double(1.0 - ldexp(1.0, -(iter + 1)));
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      Real x[W];
#pragma unroll
      for (int j = 0; j < W; ++j) x[j] = msg[j * CI + cbase + G * k];
      Real m1 = R::minr(R::absr(x[0]), R::absr(x[1]));
      Real m2 = R::maxr(R::absr(x[0]), R::absr(x[1]));
      uint32_t P = R::sw(x[0]) ^ R::sw(x[1]);
#pragma unroll
      for (int j = 2; j < W; ++j) {
        m2 = R::med3(m1, m2, R::absr(x[j]));
        m1 = R::minr(m1, R::absr(x[j]));
        P ^= R::sw(x[j]);
      }
      P ^= synbits << (31 - k);                         // (-1)^{s_c}
      Real s1 = R::flip(alpha * m1, P), s2 = R::flip(alpha * m2, P);
      R::opaque(s1);
      R::opaque(s2);
#pragma unroll
      for (int j = 0; j < W; ++j) {
        // the minimum over the other edges: min2 on the edge holding min1
        const Real o = R::flip(R::absr(x[j]) == m1 ? s2 : s1, R::sw(x[j]));
        msg[j * CI + cbase + G * k] = o;
        if constexpr (TRACE) {
          const int c = q + G * k;
          if (d == 0 && active && c < M)
            reinterpret_cast<Real*>(a.trace_c2v)[(long long)iter * M * W + c * W + j] = o;
        }
      }
    }
    __syncthreads();
    commit_prefetch();

    // ---- bit phase: marginal, hard decision, next v2c ----
    uint32_t nhb = 0;
#pragma unroll
    for (int k = 0; k < IV; ++k) {
      Real c[DV];
#pragma unroll
      for (int j = 0; j < DV; ++j) c[j] = *reinterpret_cast<const Real*>(smem + off[k][j]);
      // prefix sums in ascending check order starting from the channel LLR
      Real pre[DV + 1];
      pre[0] = Lv[k];
#pragma unroll
      for (int j = 0; j < DV; ++j) pre[j + 1] = pre[j] + c[j];
      const Real lout = pre[DV];
#pragma unroll
      for (int j = 0; j < DV; ++j) {
        Real acc = pre[j];
#pragma unroll
        for (int i = j + 1; i < DV; ++i) acc = acc + c[i];
        *reinterpret_cast<Real*>(smem + off[k][j]) = acc;   // v2c for the next iteration
      }
      nhb |= (lout > (Real)0 ? 0u : 1u) << k;
      if constexpr (TRACE) {
        const int v = q + G * k;
        if (d == 0 && active && v < N) reinterpret_cast<Real*>(a.trace_lout)[(long long)iter * N + v] = lout;
      }
    }
    hb = nhb & vmask;
    const uint32_t flips = active ? (hb ^ prevhb) : 0u;
    prevhb = hb;
    if constexpr (MODE == MODE_MAIN) {
      uint32_t carry = flips;
#pragma unroll
      for (int b = 0; b < PL; ++b) {
        const uint32_t t = cnt[b] & carry;
        cnt[b] ^= carry;
        carry = t;
      }
    }
    // residual toggles for bits whose hard decision changed
    {
      uint32_t f = flips;
      while (f) {
        const int k = __builtin_ctz(f);
        f &= f - 1u;
        const int v = q + (k << LG);
#pragma unroll
        for (int i = 0; i < DV; ++i) {
          const int c = chk[v * DV + i];
          const int ol = (d << LG) | (c & (G - 1));
          atomicXor(&resid[(c >> LG) * 2 + (ol >> 5)], 1u << (ol & 31));
        }
      }
    }
    __syncthreads();

    // ---- syndrome test of every slot ----
    uint32_t un = 0;
#pragma unroll
    for (int k = 0; k < IC; ++k) un |= resid[k * 2 + (lane >> 5)] >> (lane & 31);
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
          int32_t* r = a.records + (long long)f * a.rec_stride;
          if (need) {
            if (q == 0) {
              r[REC_SHOT] = (int32_t)shot;
              r[REC_MAIN_ITERS] = iter;
              r[REC_MAIN_CONV] = conv ? 1 : 0;
              a.keys[f] = KEY_NONE;
            }
            r[REC_HDR + KMAX + q] = (int32_t)synbits;
          }
          for (int j = 0; j < a.k; ++j) {
            uint32_t best = 0;
#pragma unroll
            for (int k = 0; k < IV; ++k) best = key[k] > best ? key[k] : best;
#pragma unroll
            for (int o = G / 2; o >= 1; o >>= 1) {
              const uint32_t other = (uint32_t)__shfl_xor((int)best, o);
              best = other > best ? other : best;
            }
            const int v = 0xffff - (int)(best & 0xffffu);
            if (need && q == (j & (G - 1))) r[REC_HDR + j] = v;
            if ((v & (G - 1)) == q) {
#pragma unroll
              for (int k = 0; k < IV; ++k)
                if (q + G * k == v) key[k] = 0u;
            }
          }
        }
      } else if constexpr (MODE == MODE_CAND) {
        // weight of the undone correction e = e' + t over the slot
        int w = __popc((hb ^ tbits) & vmask);
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) w += __shfl_xor(w, o);
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

template <typename Real, int D, int IC, int IV, int W, int DV>
static int launch_tile(int mode, bool trace, const Args& a, int grid, void* stream)
{
  using T = TileShape<D, IC, IV, W, DV>;
  const LdsLayout lay = lds_layout(sizeof(Real), W, a.CI, T::RW, a.N, DV, T::RING, T::META, T::KMAX, T::G);
  const size_t sh = lay.total;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (mode == MODE_MAIN && trace)
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, MODE_MAIN, true>), dim3(grid), dim3(64), sh, st, a);
  else if (mode == MODE_MAIN)
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, MODE_MAIN, false>), dim3(grid), dim3(64), sh, st, a);
  else if (mode == MODE_CAND)
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, MODE_CAND, false>), dim3(grid), dim3(64), sh, st, a);
  else
    hipLaunchKernelGGL((bpsf_kernel<Real, D, IC, IV, W, DV, MODE_EMIT, false>), dim3(grid), dim3(64), sh, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real, int D, int IC, int IV, int W, int DV>
static int occupancy_tile(int mode, const Args& a, int* blocks_per_cu)
{
  using T = TileShape<D, IC, IV, W, DV>;
  const LdsLayout lay = lds_layout(sizeof(Real), W, a.CI, T::RW, a.N, DV, T::RING, T::META, T::KMAX, T::G);
  hipError_t e;
  if (mode == MODE_MAIN)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bpsf_kernel<Real, D, IC, IV, W, DV, MODE_MAIN, false>, 64, lay.total);
  else if (mode == MODE_CAND)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bpsf_kernel<Real, D, IC, IV, W, DV, MODE_CAND, false>, 64, lay.total);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bpsf_kernel<Real, D, IC, IV, W, DV, MODE_EMIT, false>, 64, lay.total);
  return e == hipSuccess ? 0 : -1;
}

#define BPSF_TILE_CASE(D_, IC_, IV_, W_, DV_)                                                   \
  if (t.D == D_ && t.IC == IC_ && t.IV == IV_ && t.W == W_ && t.DV == DV_) {                    \
    if (fp64) return what == 0 ? launch_tile<double, D_, IC_, IV_, W_, DV_>(mode, trace, a, grid, st) \
                               : occupancy_tile<double, D_, IC_, IV_, W_, DV_>(mode, a, out);   \
    return what == 0 ? launch_tile<float, D_, IC_, IV_, W_, DV_>(mode, trace, a, grid, st)     \
                     : occupancy_tile<float, D_, IC_, IV_, W_, DV_>(mode, a, out);             \
  }

int tile_dispatch(int what, const TileDesc& t, bool fp64, int mode, bool trace, const Args& a, int grid,
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
