// BP-SF kernels for large irregular matrices (circuit-level detector error
// models, thousands of columns of weight 2..10 and rows of weight up to
// ~40): one decode per workgroup, float messages. Same method and arithmetic
// as bpsf_kernels.hip (paper Section II-B steps 1-4, Eq. (c2v), Algorithm 1),
// same modes and keys.
//
// Layout and schedule:
//   * checks and bits are numbered internally by weight (the host permutes
//     them at load), so the 64 rows or columns a wave handles together have
//     nearly equal weights and every loop runs to the wave's largest weight
//     (a scalar bound); results are written back in the caller's numbering,
//     and ties of the top-|Phi| selection go to the lowest index of that
//     numbering;
//   * one message per Tanner edge in LDS, edges in column-major order (the
//     edges of a bit are contiguous, by ascending check): the bit phase reads
//     and rewrites a run of consecutive cells; the check phase gathers its
//     row's cells through offsets held in registers (two 16-bit offsets per
//     word); a row's positions past its weight point at a cell of the
//     owning thread that holds +inf when read (no minimum, no sign) and takes
//     the junk written back;
//   * thread g owns the checks g + T i and the bits g + T i (T threads);
//   * u = H e and s (or s') are bit vectors in LDS; a bit whose hard decision
//     flips toggles its checks in u;
//   * an iteration is: check phase, which also compares u with s for the
//     hard decisions of the previous iteration; one barrier; the decision to
//     stop (the check phase's c2v are then dropped, the decode is over); bit
//     phase; one barrier;
//   * a failed first BP leaves a record holding its Phi; a trial rebuilds
//     s' = s + t H^T from the shot's syndrome and the columns of Phi.
#include <hip/hip_runtime.h>

#include <atomic>
#include <math.h>
#include <stdint.h>

#include "bpsf_device.h"
#include "bpsf_internal.h"
#include "bpsf_tiles.h"
#include "bpsf_sparse.h"

namespace bpsf {

namespace {

// The caller's index of my internal bit g + T i. The index passes through an
// empty asm so that the compiler does not hoist the table addresses of all
// my bits out of the task loop (they would hold 64-bit registers for the
// whole kernel).
__device__ __forceinline__ int caller_bit(const Args& a, int v)
{
  asm volatile("" : "+v"(v));
  return a.sp_cperm[v];
}

// Bit phase of one bit whose column starts at cell e0 and has w edges, for a
// wave whose largest weight in this slot is K: the marginal and the v2c of
// every edge, each summed from the channel LLR in ascending check order.
// Loads past w read +0 (the next column's cells are replaced), stores past w
// go to the junk cell. UNI: every bit of the wave has weight K (no lane has
// a position past its weight).
template <int K, bool UNI>
__device__ __forceinline__ float bit_update(float* msg, uint32_t e0, uint32_t w, float L, uint32_t junk)
{
  float cv[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float y = msg[e0 + j];
    cv[j] = (UNI || (uint32_t)j < w) ? y : 0.f;
  }
  float pre[K + 1];
  pre[0] = L;
#pragma unroll
  for (int j = 0; j < K; ++j) pre[j + 1] = pre[j] + cv[j];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    float acc = pre[j];
#pragma unroll
    for (int q = j + 1; q < K; ++q) acc = acc + cv[q];
    msg[(UNI || (uint32_t)j < w) ? e0 + j : junk] = acc;
  }
  return pre[K];
}

// Largest value of x over the wave (the same in every lane, as a scalar).
__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
  x = group_reduce(x, 64, OpMax());
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// The message cell named by half h (0: low, 1: high) of a packed word of
// 16-bit cell indices. Messages start at LDS byte 0 (the kernel has no static
// LDS, checked on the host before every launch), so the byte address is the
// index times four: one shift of a 16-bit operand, with no base to add.
__device__ __forceinline__ __attribute__((address_space(3))) float& cell_ref(unsigned char* smem, uint32_t w, int h)
{
  (void)smem;
  uint32_t b;
  if (h) {
    b = (w >> 16) << 2;
  } else {
    // the low half shifted in one instruction (the compiler rewrites the
    // mask-then-shift into two)
    asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(b) : "v"(w));
  }
  return *(__attribute__((address_space(3))) float*)(size_t)b;
}

template <int NW, int CPT, int WMAX, int BPT, int DVMAX, int MODE>
__device__ __forceinline__ void decode_sparse(const Args& a)
{
  using R = RT<float>;
  using F = SparseFamily<NW, CPT, WMAX, BPT, DVMAX>;
  constexpr int T = F::T, PL = F::PL, KMAX = F::KMAX;
  constexpr int CH = 8;   // row positions loaded together
  static_assert(WMAX % CH == 0 && CH == 8, "rows are read in chunks of 8 positions (tails of 4, 2, 1)");
  const int M = a.M, N = a.N, E = a.E;
  const SparseLayout lay = sparse_layout(E, M, NW, DVMAX, CPT);
  extern __shared__ __align__(16) unsigned char smem[];
  float* msg = reinterpret_cast<float*>(smem + lay.msg);
  uint32_t* ub = reinterpret_cast<uint32_t*>(smem + lay.ubits);
  uint32_t* sb = reinterpret_cast<uint32_t*>(smem + lay.sbits);
  uint32_t* red = reinterpret_cast<uint32_t*>(smem + lay.red);
  long long* task = reinterpret_cast<long long*>(smem + lay.task);
  uint32_t* flags = reinterpret_cast<uint32_t*>(smem + lay.flags);

  const int g = threadIdx.x;
  const uint32_t pad0 = (uint32_t)(E + DVMAX) + (uint32_t)(g * CPT);   // my pad cells, one per check slot
  const int MW = (M + 31) >> 5;              // words of a check bit vector
  const float* __restrict__ llr = reinterpret_cast<const float*>(a.llr);
  const bool adaptive = !(a.alpha > 0.0);
  const float alpha_fixed = adaptive ? 1.0f : (float)a.alpha;

  // ---- task source ----------------------------------------------------------
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
  // the workgroup's first task is its block index and the counter hands out
  // the rest after gridDim.x, so a workgroup with nothing to do leaves before
  // its set-up (small calls launch many)
  if ((long long)blockIdx.x >= n_tasks) return;
  bool first_task = true;

  // ---- per-thread constants -------------------------------------------------
  // my checks: their edges as packed 16-bit cell indices (my pad cell past
  // the weight), and the wave's largest weight
  uint32_t roff[CPT][WMAX / 2];
  uint32_t rbound[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = g + T * i;
    const uint32_t pad = (pad0 + (uint32_t)i) * 0x10001u;
#pragma unroll
    for (int j = 0; j < WMAX / 2; ++j) roff[i][j] = pad;
    uint32_t w = 0;
    if (c < M) {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(a.sp_roff) + (long long)c * (WMAX / 2);
#pragma unroll
      for (int j = 0; j < WMAX / 2; ++j) roff[i][j] = src[j];
      w = a.sp_rw[c];
    }
    rbound[i] = wave_max(w);
  }
  // my bits: first edge | weight << 16, channel LLR, and the wave's largest
  // weight per bit slot (4 bits each)
  uint32_t bw[BPT];
  float Lv[BPT];
  uint32_t wbp[(BPT + 7) / 8];
  uint32_t unim = 0;   // slots whose bits all have the wave's largest weight
  uint32_t vmask = 0;
#pragma unroll
  for (int w = 0; w < (BPT + 7) / 8; ++w) wbp[w] = 0;
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int v = g + T * i;
    bw[i] = 0;
    Lv[i] = 0.f;
    if (v < N) {
      bw[i] = a.sp_bits[v];
      Lv[i] = llr[a.sp_cperm[v]];
      vmask |= 1u << i;
    }
    const uint32_t wmax = wave_max(bw[i] >> 16), wmin = ~wave_max(~(bw[i] >> 16));
    wbp[i >> 3] |= wmax << (4 * (i & 7));
    unim |= (wmin == wmax ? 1u : 0u) << i;
  }
  // cells past the last column: read by the bit phase, never used
  for (int i = g; i < DVMAX; i += T) msg[E + i] = 0.f;

  const int rstride = a.rec_stride;
  unsigned long long st_iters = 0, st_conv = 0, st_err = 0;

  for (;;) {
    // ---- claim one task for the workgroup (thread 0 decides for everyone) ----
    __syncthreads();
    if (g == 0) {
      const long long t0 = first_task ? (long long)blockIdx.x
                                      : (long long)atomicAdd(next_ctr, 1ull) + (long long)gridDim.x;
      long long f = 0, ti = 0;
      int skip = 0;
      if (MODE != MODE_MAIN && t0 < n_tasks) {
        if (MODE == MODE_CAND) {
          if (a.flags & FLAG_PRUNE) {   // trial-major (as in the one-wave kernels)
            const long long F = n_tasks / a.n_trials;
            ti = t0 / F;
            f = t0 - ti * F;
          } else {
            f = t0 / a.n_trials;
            ti = t0 - f * a.n_trials;
          }
        } else {
          f = t0;
        }
        const unsigned long long kk = __hip_atomic_load(&a.keys[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (MODE == MODE_EMIT) {
          skip = kk == KEY_NONE;   // no trial succeeded: the first BP's output stands
          ti = skip ? 0 : (long long)((kk >> KEY_ITER_BITS) & 0xffffffffull);
        } else if (a.flags & FLAG_PRUNE) {
          skip = kk != KEY_NONE && (long long)((kk >> KEY_ITER_BITS) & 0xffffffffull) < ti;
        }
      }
      task[0] = t0;
      task[1] = f;
      task[2] = ti;
      task[3] = skip;
    }
    __syncthreads();
    first_task = false;
    const long long t = task[0];
    if (t >= n_tasks) break;
    if (task[3]) continue;
    if constexpr (MODE == MODE_EMIT) {
      if (a.trial_bits && task[1] < a.trial_bits_recs) {
        // the winner's correction as the trial kernel kept it: no decode
        const int f = (int)task[1], ti = (int)task[2];
        const int32_t* rr = a.records + (long long)f * rstride;
        const long long sh = rr[REC_SHOT];
        const uint32_t e = a.trial_bits[((long long)f * a.n_trials + ti) * T + g];
        uint8_t* out = a.corrections + sh * a.corr_stride;
#pragma unroll
        for (int i = 0; i < BPT; ++i)
          if ((vmask >> i) & 1u) out[caller_bit(a, g + T * i)] = (uint8_t)((e >> i) & 1u);
        if (g == 0) {
          const unsigned long long kk = a.keys[f];
          a.converged[sh] = 1;
          a.iterations[sh] = rr[REC_MAIN_ITERS] + (int)(kk & ((1ull << KEY_ITER_BITS) - 1ull));
        }
        continue;
      }
    }

    // ---- inputs: s into LDS bits (internal check order), u = 0 ----
    long long shot = 0;
    int rec = 0, trial = 0, main_iters = 0;
    const int32_t* r = nullptr;
    if constexpr (MODE == MODE_MAIN) {
      shot = a.shot_base + t;
    } else {
      rec = (int)task[1];
      trial = (int)task[2];
      r = a.records + (long long)rec * rstride;
      shot = r[REC_SHOT];
      main_iters = r[REC_MAIN_ITERS];
    }
    {
      const uint8_t* s = a.syndromes + shot * a.syn_stride;
      for (int c0 = 0; c0 < M; c0 += T) {
        const int c = c0 + g;
        const unsigned long long b = __ballot(c < M && (s[a.sp_rperm[c < M ? c : 0]] & 1u));
        if ((g & 63) == 0 && c < M) {
          sb[c >> 5] = (uint32_t)b;
          if ((c >> 5) + 1 < MW) sb[(c >> 5) + 1] = (uint32_t)(b >> 32);
        }
      }
      for (int i = g; i < MW; i += T) ub[i] = 0u;
    }
    uint32_t tbits = 0;
    if constexpr (MODE != MODE_MAIN) {
      // s' = s + t H^T: thread j flips the checks of Phi[j] (an internal bit
      // index) when the trial has it
      __syncthreads();
      const long long mi = shot * a.mask_stride + trial;
      const uint64_t mask = (a.flags & SPARSE_FLAG_MASKS64) ? reinterpret_cast<const uint64_t*>(a.trial_masks)[mi]
                                                             : (uint64_t)a.trial_masks[mi];
      if (g < a.k && ((mask >> g) & 1ull)) {
        const int v = r[REC_HDR + g];
        const uint32_t b = a.sp_bits[v];
        for (uint32_t e = b & 0xffffu; e < (b & 0xffffu) + (b >> 16); ++e) {
          const int c = a.sp_echk[e];
          atomicXor(&sb[c >> 5], 1u << (c & 31));
        }
      }
      for (int j = 0; j < a.k; ++j) {
        if ((mask >> j) & 1ull) {
          const int v = r[REC_HDR + j];
          if (v % T == g) tbits |= 1u << (v / T);
        }
      }
    }
    __syncthreads();
    uint32_t synbits = 0;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = g + T * i;
      if (c < M) synbits |= ((sb[c >> 5] >> (c & 31)) & 1u) << i;
    }

    // ---- fresh messages: v2c = channel LLR (c2v = 0) ----
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const uint32_t e0 = bw[i] & 0xffffu, w = bw[i] >> 16;
      for (uint32_t j = 0; j < w; ++j) msg[e0 + j] = Lv[i];
    }
    __syncthreads();

    uint32_t hb = 0, prevc = 0;
    uint32_t cnt[PL];
#pragma unroll
    for (int b = 0; b < PL; ++b) cnt[b] = 0;
    int iter = 0;
    bool conv = false;
    const int cap = MODE == MODE_MAIN ? a.max_iter : a.cand_max_iter;
    for (;;) {
      // the offsets and bounds pass through an empty asm every iteration:
      // the compiler would otherwise hoist every address and lane mask
      // derived from them out of the loop and hold it in registers for the
      // whole decode
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
#pragma unroll
        for (int j = 0; j < WMAX / 2; ++j) asm volatile("" : "+v"(roff[i][j]));
        asm volatile("" : "+v"(rbound[i]));
      }

      // ---- check phase: c2v from v2c, Eq. (c2v); and the syndrome test of
      // the last hard decisions (u against s on my checks) ----
      const float alpha = adaptive ? R::adaptive_alpha(iter + 1) : alpha_fixed;
      uint32_t unsat = 0;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int c = g + T * i;
        if (c < M) unsat |= (ub[c >> 5] >> (c & 31)) ^ (synbits >> i);
        msg[pad0 + i] = INFINITY;   // what my padded positions read
        const uint32_t rb = (uint32_t)__builtin_amdgcn_readfirstlane((int)rbound[i]);
        // two passes over the row in chunks of CH positions whose loads are
        // issued together: minima and sign parity, then the outputs; the row
        // is read twice rather than held in registers. The wave's bound need
        // not be a multiple of CH: its tail runs as chunks of 4, 2 and 1
        // positions (at most three waits for loads, not one per position).
        auto over_row = [&](auto&& chunk) {
#pragma unroll
          for (int jc = 0; jc < WMAX; jc += CH) {
            if ((uint32_t)jc + CH <= rb) {
              chunk(jc, CH);
            } else if ((uint32_t)jc < rb) {
              const uint32_t rem = rb - (uint32_t)jc;   // 1 .. CH - 1, the same in every lane
              if (rem & 4u) {
                chunk(jc, 4);
                if (rem & 2u) {
                  chunk(jc + 4, 2);
                  if (rem & 1u) chunk(jc + 6, 1);
                } else if (rem & 1u) {
                  chunk(jc + 4, 1);
                }
              } else if (rem & 2u) {
                chunk(jc, 2);
                if (rem & 1u) chunk(jc + 2, 1);
              } else {
                chunk(jc, 1);
              }
            }
          }
        };
        float m1 = INFINITY, m2 = INFINITY;
        uint32_t P = synbits << (31 - i);                  // (-1)^{s_c}
        over_row([&](const int j0, const int n) {          // positions j0 .. j0 + n - 1
          float x[CH];
#pragma unroll
          for (int q = 0; q < n; ++q) x[q] = cell_ref(smem, roff[i][(j0 + q) >> 1], (j0 + q) & 1);
#pragma unroll
          for (int q = 0; q < n; ++q) {
            m2 = R::med3(m1, m2, R::absr(x[q]));
            m1 = R::minr(m1, R::absr(x[q]));
          }
#pragma unroll
          for (int q = 0; q + 1 < n; q += 2) P = xor3(P, R::sw(x[q]), R::sw(x[q + 1]));   // two signs per op
          if (n & 1) P ^= R::sw(x[n - 1]);
        });
        float s1 = R::flip(alpha * m1, P), s2 = R::flip(alpha * m2, P);
        R::opaque(s1);
        R::opaque(s2);
        // (addresses recomputed for the second pass rather than kept)
#pragma unroll
        for (int j = 0; j < WMAX / 2; ++j) asm volatile("" : "+v"(roff[i][j]));
        over_row([&](const int j0, const int n) {
          float x[CH];
#pragma unroll
          for (int q = 0; q < n; ++q) x[q] = cell_ref(smem, roff[i][(j0 + q) >> 1], (j0 + q) & 1);
#pragma unroll
          for (int q = 0; q < n; ++q)
            cell_ref(smem, roff[i][(j0 + q) >> 1], (j0 + q) & 1) = R::flip(R::absr(x[q]) == m1 ? s2 : s1, R::sw(x[q]));
        });
      }
      const unsigned long long anyw = __ballot((unsat & 1u) != 0u);
      if ((g & 63) == 0) flags[(iter & 1) * (NW + 1) + (g >> 6)] = anyw != 0ull ? 1u : 0u;
      if constexpr (MODE == MODE_CAND) {
        // stop once a lower-index trial of the shot has succeeded (thread 0
        // reads the key for the workgroup; a stale value only stops later)
        if (g == 0) {
          uint32_t stop = 0;
          if ((a.flags & FLAG_PRUNE) && iter > 0 && (iter & 1) == 0) {
            const unsigned long long kk = __hip_atomic_load(&a.keys[rec], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = kk != KEY_NONE && (int)((kk >> KEY_ITER_BITS) & 0xffffffffull) < trial;
          }
          flags[(iter & 1) * (NW + 1) + NW] = stop;
        }
      }
      __syncthreads();
      if (iter > 0) {
        // the test of the hard decisions of iteration `iter`; stopping here
        // drops the c2v just computed
        uint32_t anyun = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) anyun |= flags[(iter & 1) * (NW + 1) + w];
        conv = anyun == 0u;
        bool stop = false;
        if constexpr (MODE == MODE_CAND) stop = flags[(iter & 1) * (NW + 1) + NW] != 0u;
        if ((conv && !(a.flags & FLAG_NO_EARLY_STOP)) || iter >= cap || stop) break;
      }

      // ---- bit phase: marginal, hard decision, next v2c (ascending checks) ----
#pragma unroll
      for (int i = 0; i < BPT; ++i) asm volatile("" : "+v"(bw[i]));
#pragma unroll
      for (int w = 0; w < (BPT + 7) / 8; ++w) asm volatile("" : "+v"(wbp[w]));
      asm volatile("" : "+v"(unim));
      const uint32_t uni = (uint32_t)__builtin_amdgcn_readfirstlane((int)unim);
      uint32_t nhb = 0;
      // one bit slot at a time, in straight-line code for the wave's largest
      // weight of the slot (a load past a bit's weight reads the next column
      // or a cell past the last one and is replaced by +0, which changes no
      // sum, so the order is the oracle's)
#pragma unroll
      for (int i = 0; i < BPT; ++i) {
        const uint32_t e0 = bw[i] & 0xffffu, w = bw[i] >> 16;
        const uint32_t wb = (uint32_t)__builtin_amdgcn_readfirstlane((int)((wbp[i >> 3] >> (4 * (i & 7))) & 15u));
        float lout;
        switch (wb) {
#define BPSF_BIT_CASE(K)                                             \
  case K:                                                            \
    lout = ((uni >> i) & 1u) ? bit_update<K, true>(msg, e0, w, Lv[i], pad0) \
                             : bit_update<K, false>(msg, e0, w, Lv[i], pad0); \
    break;
          BPSF_BIT_CASE(1) BPSF_BIT_CASE(2) BPSF_BIT_CASE(3) BPSF_BIT_CASE(4) BPSF_BIT_CASE(5)
          BPSF_BIT_CASE(6) BPSF_BIT_CASE(7) BPSF_BIT_CASE(8) BPSF_BIT_CASE(9) BPSF_BIT_CASE(10)
#undef BPSF_BIT_CASE
          default: lout = Lv[i]; break;   // a slot no bit of the wave has
        }
        nhb |= (R::nonpos_msb(lout) >> 31) << i;
      }
      const uint32_t fl = (nhb & vmask) ^ hb;
      hb = nhb & vmask;
      if constexpr (MODE == MODE_MAIN) {
        const uint32_t fc = hb ^ prevc;
        prevc = hb;
        uint32_t carry = fc;
#pragma unroll
        for (int b = 0; b < PL; ++b) {
          const uint32_t tt = cnt[b] & carry;
          cnt[b] ^= carry;
          carry = tt;
        }
      }
      // u follows the hard decisions: a flipped bit toggles its checks (the
      // check of every edge from a device table; all loads first)
      if (fl) {
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
          if ((fl >> i) & 1u) {
            const uint32_t e0 = bw[i] & 0xffffu, w = bw[i] >> 16;
            uint32_t cc[DVMAX];
#pragma unroll
            for (int j = 0; j < DVMAX; ++j) cc[j] = a.sp_echk[(uint32_t)j < w ? e0 + j : 0u];
#pragma unroll
            for (int j = 0; j < DVMAX; ++j)
              if ((uint32_t)j < w) atomicXor(&ub[cc[j] >> 5], 1u << (cc[j] & 31));
          }
        }
      }
      __syncthreads();
      ++iter;
    }

    // ---- finish ----
    if constexpr (MODE == MODE_MAIN) {
      uint8_t* out = a.corrections + shot * a.corr_stride;
#pragma unroll
      for (int i = 0; i < BPT; ++i)
        if ((vmask >> i) & 1u) out[caller_bit(a, g + T * i)] = (uint8_t)((hb >> i) & 1u);
      if (g == 0) {
        a.converged[shot] = (uint8_t)conv;
        a.iterations[shot] = iter;
        st_iters += (unsigned long long)iter;
      }
      if (a.k > 0 && (!conv || (a.flags & FLAG_FORCE_PP))) {
        // key = count << 16 | (0xffff - caller's index): largest count, then
        // lowest index of the caller's numbering
        uint32_t key[BPT];
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
          uint32_t cn = 0;
#pragma unroll
          for (int b = 0; b < PL; ++b) cn |= ((cnt[b] >> i) & 1u) << b;
          const int v = g + T * i < N ? g + T * i : N - 1;
          key[i] = ((vmask >> i) & 1u) ? ((cn << 16) | (uint32_t)(0xffff - caller_bit(a, v))) : 0u;
        }
        if (g == 0) task[1] = (long long)atomicAdd(&a.counters[CNT_FAILED], 1ull);
        __syncthreads();
        const int f = (int)task[1];
        int32_t* rr = a.records + (long long)f * rstride;
        if (g == 0) {
          rr[REC_SHOT] = (int32_t)shot;
          rr[REC_MAIN_ITERS] = iter;
          rr[REC_MAIN_CONV] = conv ? 1 : 0;
          a.keys[f] = KEY_NONE;
        }
        for (int j = 0; j < a.k; ++j) {
          uint32_t best = 0;
#pragma unroll
          for (int i = 0; i < BPT; ++i) best = key[i] > best ? key[i] : best;
          best = wg_reduce<NW>(best, OpMax(), red);
          const int vo = best ? 0xffff - (int)(best & 0xffffu) : 0;
          const int v = a.sp_cinv[vo];                     // internal index
          if (g == 0) rr[REC_HDR + j] = v;
          if (v % T == g) {
#pragma unroll
            for (int i = 0; i < BPT; ++i)
              if (g + T * i == v) key[i] = 0u;
          }
        }
      }
    } else if constexpr (MODE == MODE_CAND) {
      if (a.trial_bits && conv && rec < a.trial_bits_recs)
        a.trial_bits[((long long)rec * a.n_trials + trial) * T + g] = (hb ^ tbits) & vmask;
      const uint32_t w = wg_reduce<NW>((uint32_t)__popc((hb ^ tbits) & vmask), OpAdd(), red);
      if (g == 0) {
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
    } else {
      uint8_t* out = a.corrections + shot * a.corr_stride;
      const uint32_t e = hb ^ tbits;
#pragma unroll
      for (int i = 0; i < BPT; ++i)
        if ((vmask >> i) & 1u) out[caller_bit(a, g + T * i)] = (uint8_t)((e >> i) & 1u);
      if (g == 0) {
        a.converged[shot] = 1;
        a.iterations[shot] = main_iters + iter;
        st_iters += (unsigned long long)iter;
        if (!conv) st_err += 1;
      }
    }
  }

  if (g == 0) {
    const int sidx = MODE == MODE_MAIN ? ST_MAIN_ITERS : (MODE == MODE_CAND ? ST_CAND_ITERS : ST_EMIT_ITERS);
    if (st_iters) atomicAdd(&a.counters[sidx], st_iters);
    if (st_conv) atomicAdd(&a.counters[ST_CAND_CONV], st_conv);
    if (st_err) atomicAdd(&a.counters[ST_ERRORS], st_err);
    atomicAdd(&a.counters[ST_WAVES], 1ull);
  }
}

template <int NW, int CPT, int WMAX, int BPT, int DVMAX, int MODE>
__global__ __launch_bounds__(64 * NW) void bpsf_sparse_kernel(Args a)
{
  decode_sparse<NW, CPT, WMAX, BPT, DVMAX, MODE>(a);
}

template <int NW, int CPT, int WMAX, int BPT, int DVMAX, int MODE>
int run_sparse_mode(int what, const Args& a, size_t lds, int grid, hipStream_t st, int* out)
{
  // the row gathers address messages from LDS byte 0 (cell_ref): the kernel
  // must have no static LDS ahead of its dynamic array
  static const bool lds_at_zero = [] {
    hipFuncAttributes fa;
    return hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(bpsf_sparse_kernel<NW, CPT, WMAX, BPT, DVMAX, MODE>)) ==
               hipSuccess &&
           fa.sharedSizeBytes == 0;
  }();
  if (!lds_at_zero) return -1;
  // a workgroup may use more than 64 KiB of LDS once the kernel allows it
  // (raised once per device and size, not before every launch)
  constexpr int MAX_DEVICES = 64;
  static std::atomic<size_t> allowed[MAX_DEVICES];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::atomic<size_t>* al = dev >= 0 && dev < MAX_DEVICES ? &allowed[dev] : nullptr;
  if (!al || lds > al->load(std::memory_order_relaxed)) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(bpsf_sparse_kernel<NW, CPT, WMAX, BPT, DVMAX, MODE>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return -1;
    if (al) {
      size_t cur = al->load(std::memory_order_relaxed);
      while (lds > cur && !al->compare_exchange_weak(cur, lds, std::memory_order_relaxed)) {
      }
    }
  }
  if (what == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_sparse_kernel<NW, CPT, WMAX, BPT, DVMAX, MODE>,
                                                        64 * NW, lds) == hipSuccess ? 0 : -1;
  hipLaunchKernelGGL((bpsf_sparse_kernel<NW, CPT, WMAX, BPT, DVMAX, MODE>), dim3(grid), dim3(64 * NW), lds, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int NW, int CPT, int WMAX, int BPT, int DVMAX>
int run_sparse(int what, int mode, const Args& a, size_t lds, int grid, hipStream_t st, int* out)
{
  if (mode == MODE_MAIN) return run_sparse_mode<NW, CPT, WMAX, BPT, DVMAX, MODE_MAIN>(what, a, lds, grid, st, out);
  if (mode == MODE_CAND) return run_sparse_mode<NW, CPT, WMAX, BPT, DVMAX, MODE_CAND>(what, a, lds, grid, st, out);
  return run_sparse_mode<NW, CPT, WMAX, BPT, DVMAX, MODE_EMIT>(what, a, lds, grid, st, out);
}

}  // namespace

int sparse_count()
{
  int n = 0;
#define BPSF_SPARSE_COUNT(NW_, CPT_, WMAX_, BPT_, DVMAX_) ++n;
  BPSF_SPARSE_LIST(BPSF_SPARSE_COUNT)
#undef BPSF_SPARSE_COUNT
  return n;
}

SparseDesc sparse_desc(int fam)
{
  int i = 0;
#define BPSF_SPARSE_DESC(NW_, CPT_, WMAX_, BPT_, DVMAX_) \
  if (i++ == fam) return SparseDesc{NW_, CPT_, WMAX_, BPT_, DVMAX_};
  BPSF_SPARSE_LIST(BPSF_SPARSE_DESC)
#undef BPSF_SPARSE_DESC
  return SparseDesc{0, 0, 0, 0, 0};
}

int sparse_dispatch(int what, int fam, int mode, const Args& a, size_t lds, int grid, void* stream, int* out)
{
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int i = 0;
#define BPSF_SPARSE_CASE(NW_, CPT_, WMAX_, BPT_, DVMAX_) \
  if (i++ == fam) return run_sparse<NW_, CPT_, WMAX_, BPT_, DVMAX_>(what, mode, a, lds, grid, st, out);
  BPSF_SPARSE_LIST(BPSF_SPARSE_CASE)
#undef BPSF_SPARSE_CASE
  return -2;
}

}  // namespace bpsf
