// BP-SF kernels for codes too large for one wave: one decode per workgroup of
// NW waves (G = 64 NW lanes), with irregular row and column weights padded
// to W and DV. Same method and arithmetic as bpsf_kernels.hip (paper Section
// II-B steps 1-4, Eq. (c2v), Algorithm 1), same modes, records and keys.
//
// Layout and padding:
//   * lane g owns the block of checks c = g*IC + k (k < IC) and the bits
//     v = g + G*k (k < IV); checks are padded to MP = G*IC;
//   * messages in LDS as [edge position j][check c] (stride MP). A padded
//     position (j at or above the check's weight, or c >= M) holds +inf: it
//     never sets a minimum or a sign, and the check phase rewrites +inf there;
//   * a bit with fewer than DV checks reads its missing edges from a cell
//     that holds 0 (adding +0 changes no sum) and writes them to a per-lane
//     dummy cell;
//   * a fresh decode copies its initial v2c (the channel LLR of every edge,
//     +inf on padding) from a device table built by the host;
//   * the syndrome test, the top-|Phi| maxima and the trial weight combine
//     per-wave ballots and reductions through LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bpsf_device.h"
#include "bpsf_internal.h"
#include "bpsf_tiles.h"

namespace bpsf {

namespace {

template <typename Real, int NW, int IC, int IV, int W, int DV, int MODE>
__device__ __forceinline__ void decode_wide(const Args& a)
{
  using R = RT<Real>;
  using F = WideFamily<NW, IC, IV, W, DV>;
  constexpr int G = F::G, MP = F::MP, PL = F::PL, KMAX = F::KMAX;
  const WideLayout lay = wide_layout(sizeof(Real), W, MP, NW);
  extern __shared__ __align__(16) unsigned char smem[];
  Real* msg = reinterpret_cast<Real*>(smem + lay.msg);
  uint32_t* uw = reinterpret_cast<uint32_t*>(smem + lay.resid);
  uint32_t* red = reinterpret_cast<uint32_t*>(smem + lay.red);
  long long* task = reinterpret_cast<long long*>(smem + lay.task);
  uint32_t* flags = reinterpret_cast<uint32_t*>(smem + lay.flags);

  const int g = threadIdx.x;          // lane of the decode
  const int M = a.M, N = a.N;
  const Real* __restrict__ llr = reinterpret_cast<const Real*>(a.llr);
  const Real* __restrict__ init = reinterpret_cast<const Real*>(a.edge_init);
  const bool adaptive = !(a.alpha > 0.0);
  const Real alpha_fixed = R::from_double(adaptive ? 1.0 : a.alpha);
  const Real INF = (Real)INFINITY;

  // ---- task source ----------------------------------------------------------
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
  // the workgroup's first task is its block index and the counter hands out
  // the rest after gridDim.x, so a workgroup with nothing to do leaves before
  // its set-up (small calls launch many)
  if ((long long)blockIdx.x >= n_tasks) return;
  bool first_task = true;

  // ---- per-lane constants ---------------------------------------------------
  const uint32_t zero_cell = lay.zero;
  const uint32_t dummy_cell = lay.dummy + (uint32_t)sizeof(Real) * (uint32_t)g;   // write-only
  uint32_t off[IV][DV];        // byte offsets of my bits' edges (reads)
  uint64_t emask = 0;          // edge (k, j) is a real edge
  uint32_t vmask = 0;
  Real Lv[IV];
#pragma unroll
  for (int k = 0; k < IV; ++k) {
    const int v = g + G * k;
    Lv[k] = (Real)0;
#pragma unroll
    for (int j = 0; j < DV; ++j) off[k][j] = zero_cell;
    if (v < N) {
      vmask |= 1u << k;
      Lv[k] = llr[v];
#pragma unroll
      for (int j = 0; j < DV; ++j) {
        const int c = a.var_chk[v * DV + j];
        if (c != 0xffff) {
          off[k][j] = lay.msg + (uint32_t)sizeof(Real) * (uint32_t)(a.var_pos[v * DV + j] * MP + c);
          emask |= 1ull << (k * DV + j);
        }
      }
    }
  }
  // row weights of my check items (0 for padding checks)
  uint32_t rw[IC];
#pragma unroll
  for (int k = 0; k < IC; ++k) {
    const int c = g * IC + k;
    rw[k] = c < M ? (uint32_t)a.row_w[c] : 0u;
  }
  for (int i = g; i < MP; i += G) uw[i] = 0u;
  if (g == 0) *reinterpret_cast<Real*>(smem + zero_cell) = (Real)0;

  const int rstride = a.rec_stride;

  uint32_t prevt = 0;                 // hard decisions u was last toggled to
  unsigned long long st_iters = 0, st_conv = 0, st_err = 0;

  for (;;) {
    // ---- claim one task for the workgroup; thread 0 also resolves the
    // record and reads its key, so every decision below is the same in
    // every thread (a key read per thread could differ under concurrent
    // updates and split the workgroup's barriers)
    __syncthreads();
    if (g == 0) {
      const long long t0 = first_task ? (long long)blockIdx.x
                                      : (long long)atomicAdd(next_ctr, 1ull) + (long long)gridDim.x;
      long long f = 0, ti = 0;
      unsigned long long kk = KEY_NONE;
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
        if (a.rec_list) f = a.rec_list[f];
        kk = __hip_atomic_load(&a.keys[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

    // ---- inputs ----
    uint32_t synbits = 0, tbits = 0;
    long long shot = 0;
    int rec = 0, trial = 0, main_iters = 0;
    if constexpr (MODE == MODE_MAIN) {
      shot = a.task_shot ? (long long)a.task_shot[t] : a.shot_base + t;
      const uint8_t* s = a.syndromes + shot * a.syn_stride;
#pragma unroll
      for (int k = 0; k < IC; ++k) {
        const int c = g * IC + k;
        if (c < M) synbits |= ((uint32_t)s[c] & 1u) << k;
      }
    } else {
      const long long f = task[1], ti = task[2];
      const int32_t* r = a.records + f * (long long)rstride;
      shot = r[REC_SHOT];
      main_iters = r[REC_MAIN_ITERS];
      const uint32_t mask = a.trial_masks[shot * a.mask_stride + ti];
      synbits = (uint32_t)r[REC_HDR + g];
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        if (j < a.k && ((mask >> j) & 1u)) {
          const uint32_t tw = (uint32_t)r[REC_HDR + G + j * G + g];
          synbits ^= tw & 0xffffu;
          const uint32_t vi = tw >> 16;
          if (vi) tbits |= 1u << (vi - 1u);
        }
      }
      rec = (int)f;
      trial = (int)ti;
    }

    // ---- fresh messages: v2c = channel LLR (c2v = 0), +inf on padding ----
    for (int i = g; i < W * MP; i += G) msg[i] = init[i];
    __syncthreads();

    uint32_t prevc = 0, hb = 0;
    uint32_t cnt[PL];
#pragma unroll
    for (int b = 0; b < PL; ++b) cnt[b] = 0;
    int iter = 0;
    bool conv = false;
    const int cap = MODE == MODE_MAIN ? a.max_iter : a.cand_max_iter;
    for (;;) {
      // ---- check phase: c2v from v2c, Eq. (c2v) ----
      const Real alpha = adaptive ? R::adaptive_alpha(iter + 1) : alpha_fixed;
      {
        const int cb = g * IC;
        Real x[2][W];
#pragma unroll
        for (int j = 0; j < W; ++j) x[0][j] = msg[j * MP + cb];
#pragma unroll
        for (int k = 0; k < IC; ++k) {
          Real (&xc)[W] = x[k & 1];
          if (k + 1 < IC) {
#pragma unroll
            for (int j = 0; j < W; ++j) x[(k + 1) & 1][j] = msg[j * MP + cb + k + 1];
          }
          Real m1 = R::minr(R::absr(xc[0]), R::absr(xc[1]));
          Real m2 = R::maxr(R::absr(xc[0]), R::absr(xc[1]));
#pragma unroll
          for (int j = 2; j < W; ++j) {
            m2 = R::med3(m1, m2, R::absr(xc[j]));
            m1 = R::minr(m1, R::absr(xc[j]));
          }
          // sign parity, (-1)^{s_c} included, in bit 31; two signs per op
          // (padding holds +inf, which adds no sign)
          uint32_t P = synbits << (31 - k);
#pragma unroll
          for (int j = 0; j + 1 < W; j += 2) P = xor3(P, R::sw(xc[j]), R::sw(xc[j + 1]));
          if constexpr (W % 2 != 0) P ^= R::sw(xc[W - 1]);
          Real s1 = R::flip(alpha * m1, P), s2 = R::flip(alpha * m2, P);
          R::opaque(s1);
          R::opaque(s2);
#pragma unroll
          for (int j = 0; j < W; ++j) {
            const Real o = R::flip(R::absr(xc[j]) == m1 ? s2 : s1, R::sw(xc[j]));
            msg[j * MP + cb + k] = (uint32_t)j < rw[k] ? o : INF;
          }
        }
      }
      __syncthreads();

      // ---- bit phase ----
      uint32_t nhb = 0;
      {
        Real cv[IV][DV];
#pragma unroll
        for (int k = 0; k < IV; ++k)
#pragma unroll
          for (int j = 0; j < DV; ++j) cv[k][j] = *reinterpret_cast<const Real*>(smem + off[k][j]);
#pragma unroll
        for (int k = IV - 1; k >= 0; --k) {
          Real pre[DV + 1];
          pre[0] = Lv[k];
#pragma unroll
          for (int j = 0; j < DV; ++j) pre[j + 1] = pre[j] + cv[k][j];
          const Real lout = pre[DV];
#pragma unroll
          for (int j = 0; j < DV; ++j) {
            Real acc = pre[j];
#pragma unroll
            for (int i = j + 1; i < DV; ++i) acc = acc + cv[k][i];
            const uint32_t o = ((emask >> (k * DV + j)) & 1ull) ? off[k][j] : dummy_cell;
            *reinterpret_cast<Real*>(smem + o) = acc;
          }
          nhb = __builtin_amdgcn_alignbit(nhb, R::nonpos_msb(lout), 31);
        }
      }
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
      {
        uint32_t fl = hb ^ prevt;
        prevt = hb;
        while (fl) {
          const int k = __builtin_ctz(fl);
          fl &= fl - 1u;
          const int v = g + G * k;
          // all the bit's checks are loaded before the first toggle
          int cs[DV];
#pragma unroll
          for (int j = 0; j < DV; ++j) cs[j] = a.var_chk[v * DV + j];
#pragma unroll
          for (int j = 0; j < DV; ++j)
            if (cs[j] != 0xffff) atomicXor(&uw[cs[j]], 1u);
        }
      }
      __syncthreads();

      // ---- syndrome test over the whole decode ----
      uint32_t un = 0;
#pragma unroll
      for (int k = 0; k < IC; ++k) un |= uw[g * IC + k] ^ (synbits >> k);
      un &= 1u;
      const unsigned long long ub = __ballot(un != 0u);
      if ((g & 63) == 0) flags[(iter & 1) * (NW + 1) + (g >> 6)] = ub != 0ull ? 1u : 0u;
      if constexpr (MODE == MODE_CAND) {
        // stop once a lower-index trial of the shot has succeeded (thread 0
        // reads the key for the workgroup; a stale value only stops later)
        if (g == 0) {
          uint32_t stop = 0;
          if ((a.flags & FLAG_PRUNE) && (iter & 1) == 1) {
            const unsigned long long kk = __hip_atomic_load(&a.keys[rec], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            stop = kk != KEY_NONE && (int)((kk >> KEY_ITER_BITS) & 0xffffffffull) < trial;
          }
          flags[(iter & 1) * (NW + 1) + NW] = stop;
        }
      }
      __syncthreads();
      uint32_t anyun = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) anyun |= flags[(iter & 1) * (NW + 1) + w];
      conv = anyun == 0u;
      bool stop = false;
      if constexpr (MODE == MODE_CAND) stop = flags[(iter & 1) * (NW + 1) + NW] != 0u;
      ++iter;
      if ((conv && !(a.flags & FLAG_NO_EARLY_STOP)) || iter >= cap || stop) break;
    }

    // ---- finish ----
    if constexpr (MODE == MODE_MAIN) {
      uint8_t* out = a.corrections + shot * a.corr_stride;
#pragma unroll
      for (int k = 0; k < IV; ++k)
        if ((vmask >> k) & 1u) out[g + G * k] = (uint8_t)((hb >> k) & 1u);
      if (g == 0) {
        a.converged[shot] = (uint8_t)conv;
        a.iterations[shot] = iter;
        st_iters += (unsigned long long)iter;
      }
      if (a.k > 0 && (!conv || (a.flags & FLAG_FORCE_PP))) {
        uint32_t key[IV];
#pragma unroll
        for (int k = 0; k < IV; ++k) {
          uint32_t cn = 0;
#pragma unroll
          for (int b = 0; b < PL; ++b) cn |= ((cnt[b] >> k) & 1u) << b;
          key[k] = ((vmask >> k) & 1u) ? ((cn << 16) | (uint32_t)(0xffff - (g + G * k))) : 0u;
        }
        if (g == 0) {
          int f = (int)atomicAdd(&a.counters[CNT_FAILED], 1ull);
          if (a.rec_list) {
            const int i = f;
            f = (int)atomicAdd(a.rec_alloc, 1ull);
            a.rec_list[i] = f;
          }
          task[1] = f;
        }
        __syncthreads();
        const int f = (int)task[1];
        int32_t* r = a.records + (long long)f * rstride;
        if (g == 0) {
          r[REC_SHOT] = (int32_t)shot;
          r[REC_MAIN_ITERS] = iter;
          r[REC_MAIN_CONV] = conv ? 1 : 0;
          a.keys[f] = KEY_NONE;
        }
        r[REC_HDR + g] = (int32_t)synbits;
        for (int j = 0; j < a.k; ++j) {
          uint32_t best = 0;
#pragma unroll
          for (int k = 0; k < IV; ++k) best = key[k] > best ? key[k] : best;
          best = wg_reduce<NW>(best, OpMax(), red);
          const int v = best ? 0xffff - (int)(best & 0xffffu) : 0;
          uint32_t tw = 0;
#pragma unroll
          for (int i = 0; i < DV; ++i) {
            const int c = a.var_chk[v * DV + i];
            if (c != 0xffff && c / IC == g) tw ^= 1u << (c - g * IC);
          }
          if (v % G == g) tw |= (uint32_t)(v / G + 1) << 16;
          r[REC_HDR + G + j * G + g] = (int32_t)tw;
          if (g == 0) r[REC_HDR + G + a.k * G + j] = v;
          if (v % G == g) {
#pragma unroll
            for (int k = 0; k < IV; ++k)
              if (g + G * k == v) key[k] = 0u;
          }
        }
      }
    } else if constexpr (MODE == MODE_CAND) {
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
      for (int k = 0; k < IV; ++k)
        if ((vmask >> k) & 1u) out[g + G * k] = (uint8_t)((e >> k) & 1u);
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

// The float trial and re-run kernels are held to three waves per SIMD (168
// VGPRs, a few bytes of scratch outside the iteration loop): four workgroups
// of three waves per CU instead of two, as the LDS allows. The first-BP kernel
// would spill inside its loop and stays at two.
template <typename Real, int NW, int IC, int IV, int W, int DV, int MODE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 && MODE != MODE_MAIN ? 3 : 1)))
void bpsf_wide_kernel(Args a)
{
  decode_wide<Real, NW, IC, IV, W, DV, MODE>(a);
}

template <typename Real, int NW, int IC, int IV, int W, int DV>
int run_wide(int what, int mode, const Args& a, size_t lds, int grid, hipStream_t st, int* out)
{
  if (what == 1) {
    hipError_t e;
    if (mode == MODE_MAIN)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_wide_kernel<Real, NW, IC, IV, W, DV, MODE_MAIN>,
                                                       64 * NW, lds);
    else if (mode == MODE_CAND)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_wide_kernel<Real, NW, IC, IV, W, DV, MODE_CAND>,
                                                       64 * NW, lds);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bpsf_wide_kernel<Real, NW, IC, IV, W, DV, MODE_EMIT>,
                                                       64 * NW, lds);
    return e == hipSuccess ? 0 : -1;
  }
  if (mode == MODE_MAIN)
    hipLaunchKernelGGL((bpsf_wide_kernel<Real, NW, IC, IV, W, DV, MODE_MAIN>), dim3(grid), dim3(64 * NW), lds, st, a);
  else if (mode == MODE_CAND)
    hipLaunchKernelGGL((bpsf_wide_kernel<Real, NW, IC, IV, W, DV, MODE_CAND>), dim3(grid), dim3(64 * NW), lds, st, a);
  else
    hipLaunchKernelGGL((bpsf_wide_kernel<Real, NW, IC, IV, W, DV, MODE_EMIT>), dim3(grid), dim3(64 * NW), lds, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int wide_count()
{
  int n = 0;
#define BPSF_WIDE_COUNT(NW_, IC_, IV_, W_, DV_) ++n;
  BPSF_WIDE_LIST(BPSF_WIDE_COUNT)
#undef BPSF_WIDE_COUNT
  return n;
}

WideDesc wide_desc(int fam)
{
  int i = 0;
#define BPSF_WIDE_DESC(NW_, IC_, IV_, W_, DV_) \
  if (i++ == fam) return WideDesc{NW_, IC_, IV_, W_, DV_};
  BPSF_WIDE_LIST(BPSF_WIDE_DESC)
#undef BPSF_WIDE_DESC
  return WideDesc{0, 0, 0, 0, 0};
}

int wide_dispatch(int what, int fam, bool fp64, int mode, const Args& a, size_t lds, int grid, void* stream, int* out)
{
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int i = 0;
#define BPSF_WIDE_CASE(NW_, IC_, IV_, W_, DV_)                                                   \
  if (i++ == fam) {                                                                              \
    return fp64 ? run_wide<double, NW_, IC_, IV_, W_, DV_>(what, mode, a, lds, grid, st, out)   \
                : run_wide<float, NW_, IC_, IV_, W_, DV_>(what, mode, a, lds, grid, st, out);   \
  }
  BPSF_WIDE_LIST(BPSF_WIDE_CASE)
#undef BPSF_WIDE_CASE
  return -2;
}

}  // namespace bpsf
