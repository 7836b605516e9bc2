// Host runtime of the BP-SF library: code loading (edge layouts), parameter
// checks, channel LLRs, trial-vector tables, scratch management and the launch
// sequence of the three decode phases. C ABI declared in include/bpsf.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bpsf.h"
#include "bpsf_internal.h"
#include "bpsf_tiles.h"
#include "bpsf_sparse.h"
#include "bpsf_sparse_layout.h"

using namespace bpsf;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

int bpsf::report_error(int code, const char* msg)
{
  g_err = msg;
  return code;
}

namespace {

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(BPSF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)


struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  // grow-only, by at least half again and to at least 1 MiB (at most `most`
  // unless `want` is more), so calls whose sizes creep up reallocate (and
  // wait for the device to free the old buffer) only a few times; contents
  // are not preserved
  int ensure(size_t want, size_t most = SIZE_MAX)
  {
    if (want <= bytes) return 0;
    const size_t grown = std::max(want, std::min(std::max(bytes + bytes / 2, (size_t)1 << 20), most));
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    if (grown > want && hipMalloc(&p, grown) == hipSuccess) {
      bytes = grown;
      return 0;
    }
    if (hipMalloc(&p, want) != hipSuccess) { p = nullptr; return -1; }
    bytes = want;
    return 0;
  }
};

}  // namespace

struct bpsf_code_s {
  int device = 0;
  int M = 0, N = 0, E = 0, W = 0, DV = 0;   // W, DV: table widths (padded for wide codes)
  int rw_max = 0, cw_max = 0;               // largest row and column weight
  int cus = 0;
  size_t lds_max = 0;                       // LDS bytes a workgroup may use
  DevBuf var_chk, var_pos, ell_col;
  // layered schedule (one-wave codes): layer of every check, bit of every
  // (check, position), number of layers (0: more than the kernels take)
  DevBuf check_layer, ell16;
  int n_layers = 0;
  // codes too large for one wave, or with irregular weights: a wide family
  int wide = -1;
  DevBuf row_w, init32, init64;
  // large irregular matrices: a sparse family (float messages only)
  int sparse = -1;
  int sp_cells = 0;          // message cells (edges plus column padding)
  DevBuf sp_roff, sp_rw, sp_bits, sp_echk, sp_rperm, sp_cperm, sp_cinv;

  std::vector<int32_t> ell_host;
  // channel LLR cache
  std::vector<double> priors;
  bool uniform = false;       // every prior equal (the LLR is then a kernel scalar)
  double llr_uniform = 0.0;
  DevBuf llr32, llr64;
  // trial masks cache
  int masks_k = -1, masks_mode = -1, masks_wmax = -1, n_trials = 0;
  // the caller's trial list (BPSF_TRIALS_TABLE)
  const uint32_t* table = nullptr;   // 32-bit masks, or 64-bit ones when table64
  int64_t table_n = 0, table_stride = 0;
  bool table64 = false;
  DevBuf masks;
  // scratch
  DevBuf records, keys, counters;
  DevBuf trial_bits;          // kept corrections of converged trials (single-code calls)
  unsigned long long* last_counters = nullptr;   // counters of the last decode call (its scratch)
  int tuned_D = 0;            // decodes per wave (0: the most that fit)
  int tuned_wpc = 0;          // resident waves per CU of the persistent grids (0: as many as fit)
  // optional per-phase timing: events[i] marks the boundary before phase i
  bool timing = false;
  bool timed_last = false;
  int timed_phases = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::mutex mu;
  ~bpsf_code_s()
  {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

// Does the code fit family `fam` at D decodes per wave?
bool tile_fits(const bpsf_code_s* c, int fam, int D)
{
  const FamilyDesc f = family_desc(fam);
  if (f.W != c->W || f.DV != c->DV) return false;
  if (D < 1 || D > MAX_D || (D & (D - 1))) return false;
  const int G = 64 / D;
  return c->M <= G * f.IC && c->N <= G * f.IV && c->N * f.DV <= 65535;
}

// A call takes the family with the fewest items per lane, at its most
// decodes per wave D, when it has at most SMALL_CALL_SHOTS_PER_D * D shots:
// such calls do not fill the GPU, so their time is the iterations of one
// decode, and one iteration of a wave is about twice as fast with a third of
// the items. Measured call times: on [[144]] (D = 2 there) the small family
// is faster up to about 16k shots, on [[288]] (D = 1) about as fast at 4k.
constexpr int64_t SMALL_CALL_SHOTS_PER_D = 4096;
// The same for mixed calls, whose batches come from a serving loop under load
// (at 3x10^6 shots/s offered, 3k-shot batches of five codes were slower on
// the small family: p99 2.1 ms against 1.5 ms).
constexpr int64_t SMALL_MIX_SHOTS_PER_D = 2048;
constexpr int64_t SMALL_CALL_SHOTS = SMALL_CALL_SHOTS_PER_D * MAX_D;   // the most any code can use
// Calls of at most this many shots per decode slot of a wave take tasks D at
// a time instead of 2D, so all the trials of their few failed shots run at
// once; measured on [[144]] (small family, D = 2): 256 shots 185 -> 164 us,
// 1024 shots 201 -> 188 us, while 2048 and 4096 shots were slower with D.
constexpr int64_t SMALL_CHUNK_SHOTS_PER_D = 512;

// Edges a lane of family `fam` works on per iteration.
int family_items(int fam)
{
  const FamilyDesc f = family_desc(fam);
  return f.IC * f.W + f.IV * f.DV;
}

// Tile of a call of `shots` shots (a forced D takes the family with the
// fewest items per lane that fits at D; a call of at most per_d x D shots that
// family at its most decodes per wave D), or, for shots < 0 (the default of
// mixed handles, traces) and larger calls, the first family the code fits, at
// the most decodes per wave (the handle's tuned or forced D when set).
int pick_tile(const bpsf_code_s* c, TileDesc* out, int64_t shots = -1, int64_t per_d = SMALL_CALL_SHOTS_PER_D)
{
  if (shots >= 0) {
    int best = -1, best_D = 0;
    for (int fam = 0; fam < family_count(); ++fam) {
      int D = 0;
      if (c->tuned_D > 0) {
        if (tile_fits(c, fam, c->tuned_D)) D = c->tuned_D;
      } else {
        for (int d = MAX_D; d >= 1 && !D; d >>= 1)
          if (tile_fits(c, fam, d)) D = d;
      }
      if (D && (best < 0 || family_items(fam) < family_items(best))) {
        best = fam;
        best_D = D;
      }
    }
    if (best < 0) return -1;
    if (c->tuned_D > 0 || shots <= per_d * best_D) {
      *out = TileDesc{best, best_D};
      return 0;
    }
  }
  for (int fam = 0; fam < family_count(); ++fam) {
    if (c->tuned_D > 0 && tile_fits(c, fam, c->tuned_D)) {
      *out = TileDesc{fam, c->tuned_D};
      return 0;
    }
    for (int D = MAX_D; D >= 1; D >>= 1)
      if (tile_fits(c, fam, D)) {
        *out = TileDesc{fam, D};
        return 0;
      }
  }
  return -1;
}

size_t tile_lds(const bpsf_code_s* c, const TileDesc& t, bool fp64, bool uniform, bool layered = false)
{
  const FamilyDesc f = family_desc(t.fam);
  return lds_layout(fp64 ? 8 : 4, f.W, 64 * f.IC, c->M, c->N, f.DV, t.D, uniform, RING_META, layered, f.IV).total;
}

// Trial vectors of Algorithm 1 as k-bit masks over Phi, in trial order.
std::vector<uint32_t> trial_masks(int k, int mode, int w_max)
{
  std::vector<uint32_t> m;
  if (k <= 0) return m;
  if (mode == BPSF_TRIALS_ALL_SUBSETS) {
    m.resize((size_t)1 << k);
    for (size_t i = 0; i < m.size(); ++i) m[i] = (uint32_t)i;
    return m;
  }
  for (int w = 1; w <= w_max; ++w) {
    std::vector<int> pos(w);
    for (int j = 0; j < w; ++j) pos[j] = j;
    for (;;) {
      uint32_t x = 0;
      for (int j = 0; j < w; ++j) x |= 1u << pos[j];
      m.push_back(x);
      int j = w - 1;
      while (j >= 0 && pos[j] == k - w + j) --j;
      if (j < 0) break;
      ++pos[j];
      for (int i = j + 1; i < w; ++i) pos[i] = pos[i - 1] + 1;
    }
  }
  return m;
}

int check_params(const bpsf_params* p)
{
  if (!p) return fail(BPSF_EINVAL, "params is NULL");
  if (p->max_iter < 1 || p->max_iter > 255) return fail(BPSF_EINVAL, "max_iter must be in 1..255");
  if (p->k < 0 || p->k > (p->cand_mode == BPSF_TRIALS_TABLE ? 64 : 16))
    return fail(BPSF_EINVAL, "k must be in 0..16 (0..64 with BPSF_TRIALS_TABLE)");
  if (p->k > 0 && (p->cand_max_iter < 1 || p->cand_max_iter >= (1 << KEY_ITER_BITS)))
    return fail(BPSF_EINVAL, "cand_max_iter must be in 1..4095");
  if (p->cand_mode != BPSF_TRIALS_ALL_SUBSETS && p->cand_mode != BPSF_TRIALS_WEIGHT_LE &&
      p->cand_mode != BPSF_TRIALS_TABLE)
    return fail(BPSF_EINVAL, "unknown cand_mode");
  if (p->k > 0 && p->cand_mode == BPSF_TRIALS_WEIGHT_LE && (p->w_max < 1 || p->w_max > p->k))
    return fail(BPSF_EINVAL, "w_max must be in 1..k");
  if (p->select_mode != BPSF_SELECT_MIN_WEIGHT && p->select_mode != BPSF_SELECT_FIRST)
    return fail(BPSF_EINVAL, "unknown select_mode");
  if ((p->flags & BPSF_FLAG_PRUNE) && p->select_mode != BPSF_SELECT_FIRST)
    return fail(BPSF_EINVAL, "BPSF_FLAG_PRUNE needs BPSF_SELECT_FIRST");
  if (!(p->alpha >= 0.0) || !isfinite(p->alpha)) return fail(BPSF_EINVAL, "alpha must be finite and >= 0");
  if (p->flags & ~(BPSF_FLAG_NO_EARLY_STOP | BPSF_FLAG_FORCE_PP | BPSF_FLAG_PRUNE | BPSF_FLAG_LAYERED))
    return fail(BPSF_EINVAL, "unknown flags");
  if (p->precision != BPSF_PREC_FP32 && p->precision != BPSF_PREC_FP64) return fail(BPSF_EINVAL, "unknown precision");
  return 0;
}

// The handle's device tables (LLRs, trial masks) are rewritten only after the
// work already enqueued on the call's stream has finished: a decode still
// queued there reads them. (The rewrite itself is a synchronous copy.)
int drain_stream(void* stream)
{
  HIP_OK(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  return 0;
}

// Channel LLRs l_v = log((1 - p_v) / p_v) (Section II-B step 1), in double on
// the host, then stored on the device in float and double.
int update_llr(bpsf_code_s* c, const double* priors, void* stream)
{
  if (!priors) return fail(BPSF_EINVAL, "priors is NULL");
  if (!c->priors.empty() && memcmp(c->priors.data(), priors, sizeof(double) * (size_t)c->N) == 0) return 0;
  std::vector<double> l64((size_t)c->N);
  std::vector<float> l32((size_t)c->N);
  for (int v = 0; v < c->N; ++v) {
    const double p = priors[v];
    if (!(p > 0.0 && p < 1.0)) return fail(BPSF_EINVAL, "priors[%d] = %g is not in (0, 1)", v, p);
    l64[v] = log((1.0 - p) / p);
    l32[v] = (float)l64[v];
  }
  if (!c->priors.empty()) {
    int rc = drain_stream(stream);
    if (rc) return rc;
  }
  if (c->llr64.ensure(sizeof(double) * (size_t)c->N) || c->llr32.ensure(sizeof(float) * (size_t)c->N))
    return fail(BPSF_ENOMEM, "LLR buffers");
  HIP_OK(hipMemcpy(c->llr64.p, l64.data(), sizeof(double) * (size_t)c->N, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(c->llr32.p, l32.data(), sizeof(float) * (size_t)c->N, hipMemcpyHostToDevice));
  if (c->wide >= 0) {
    // initial v2c of every edge position of every (padded) check: the
    // channel LLR of the edge's bit, +inf where the row has no edge
    const WideDesc d = wide_desc(c->wide);
    const size_t MP = (size_t)64 * d.NW * d.IC, n = (size_t)c->W * MP;
    std::vector<double> i64(n, HUGE_VAL);
    std::vector<float> i32(n, HUGE_VALF);
    for (int r = 0; r < c->M; ++r)
      for (int j = 0; j < c->W; ++j) {
        const int v = c->ell_host[(size_t)r * c->W + j];
        if (v >= 0) {
          i64[(size_t)j * MP + r] = l64[v];
          i32[(size_t)j * MP + r] = l32[v];
        }
      }
    if (c->init64.ensure(sizeof(double) * n) || c->init32.ensure(sizeof(float) * n))
      return fail(BPSF_ENOMEM, "initial message tables");
    HIP_OK(hipMemcpy(c->init64.p, i64.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->init32.p, i32.data(), sizeof(float) * n, hipMemcpyHostToDevice));
  }
  c->priors.assign(priors, priors + c->N);
  c->uniform = true;
  for (int v = 1; v < c->N; ++v)
    if (priors[v] != priors[0]) c->uniform = false;
  c->llr_uniform = l64[0];
  return 0;
}

int update_masks(bpsf_code_s* c, const bpsf_params* p, void* stream)
{
  if (p->cand_mode == BPSF_TRIALS_TABLE) {
    if (p->k > 0 && !c->table) return fail(BPSF_EINVAL, "BPSF_TRIALS_TABLE without a trial table on the code");
    return 0;
  }
  const int wm = p->cand_mode == BPSF_TRIALS_WEIGHT_LE ? p->w_max : 0;
  if (c->masks_k == p->k && c->masks_mode == p->cand_mode && c->masks_wmax == wm) return 0;
  std::vector<uint32_t> m = trial_masks(p->k, p->cand_mode, wm);
  if (c->masks_k >= 0) {
    int rc = drain_stream(stream);
    if (rc) return rc;
  }
  c->n_trials = (int)m.size();
  if (!m.empty()) {
    if (c->masks.ensure(sizeof(uint32_t) * m.size())) return fail(BPSF_ENOMEM, "trial mask table");
    HIP_OK(hipMemcpy(c->masks.p, m.data(), sizeof(uint32_t) * m.size(), hipMemcpyHostToDevice));
  }
  c->masks_k = p->k;
  c->masks_mode = p->cand_mode;
  c->masks_wmax = wm;
  return 0;
}

// Resident blocks per CU of a kernel at an LDS size (memoized: the answer
// depends only on the kernel, the LDS bytes and the device).
int occupancy(bool mixed, const TileDesc& t, bool fp64, bool uniform, int mode, size_t lds, const Args* a,
              const MixArgs* m, int* out, bool layered = false, bool small_mix = false)
{
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, int, int, size_t, int>, int> memo;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(dev, (int)mixed, t.fam, mixed ? (int)small_mix : t.D, (int)fp64 * 2 + (int)uniform,
                                   mode, lds, (int)layered);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) {
      *out = it->second;
      return 0;
    }
  }
  int n = 0;
  const int rc = mixed ? mixed_dispatch(1, t.fam, fp64, uniform, small_mix, mode, *m, lds, 0, nullptr, &n)
                       : tile_dispatch(1, t, fp64, uniform, mode, false, *a, lds, 0, nullptr, &n, layered);
  if (rc || n < 1) return -1;
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = n;
  *out = n;
  return 0;
}

struct Plan {
  TileDesc tile;
  int wide = -1;     // wide family of the code, or -1
  int sparse = -1;   // sparse family of the code, or -1
  Args args;
  size_t lds;
  int grid[3];
};

// Whether a call leaves out the empty trial: all subsets of Phi, trials only
// after a failed first BP (no FORCE_PP), a stop at the first success of a run
// (no NO_EARLY_STOP), and trials no longer than the first BP.
bool empty_trial_skipped(const bpsf_params* p)
{
  return p->cand_mode == BPSF_TRIALS_ALL_SUBSETS && p->k > 0 &&
         !(p->flags & (BPSF_FLAG_FORCE_PP | BPSF_FLAG_NO_EARLY_STOP)) && p->cand_max_iter <= p->max_iter;
}

// Code, geometry and parameter fields of a launch's Args (no problem
// buffers, no scratch).
int fill_code_args(const bpsf_code_s* c, const bpsf_params* p, const TileDesc& t, Args* out)
{
  if (p->k > c->N) return fail(BPSF_EINVAL, "k = %d exceeds the %d bits of the code", p->k, c->N);
  const int G = c->wide >= 0 ? 64 * wide_desc(c->wide).NW : 64 / t.D;   // lanes of a decode (one-wave, wide)
  Args& a = *out;
  memset(&a, 0, sizeof a);
  a.M = c->M;
  a.N = c->N;
  a.D = t.D;
  a.var_chk = static_cast<const uint16_t*>(c->var_chk.p);
  a.var_pos = static_cast<const uint8_t*>(c->var_pos.p);
  a.ell_col = static_cast<const int32_t*>(c->ell_col.p);
  a.llr = p->precision == BPSF_PREC_FP64 ? c->llr64.p : c->llr32.p;
  a.llr_uniform = c->llr_uniform;
  a.row_w = static_cast<const uint8_t*>(c->row_w.p);
  a.edge_init = p->precision == BPSF_PREC_FP64 ? c->init64.p : c->init32.p;
  a.check_layer = static_cast<const uint8_t*>(c->check_layer.p);
  a.ell16 = static_cast<const uint16_t*>(c->ell16.p);
  a.n_layers = c->n_layers;
  a.E = c->sparse >= 0 ? c->sp_cells : c->E;   // the sparse kernels size their message cells by it
  a.sp_roff = static_cast<const uint16_t*>(c->sp_roff.p);
  a.sp_rw = static_cast<const uint8_t*>(c->sp_rw.p);
  a.sp_bits = static_cast<const uint32_t*>(c->sp_bits.p);
  a.sp_echk = static_cast<const uint16_t*>(c->sp_echk.p);
  a.sp_rperm = static_cast<const uint16_t*>(c->sp_rperm.p);
  a.sp_cperm = static_cast<const uint16_t*>(c->sp_cperm.p);
  a.sp_cinv = static_cast<const uint16_t*>(c->sp_cinv.p);
  a.syn_stride = c->M;
  a.corr_stride = c->N;
  a.max_iter = p->max_iter;
  a.cand_max_iter = p->k > 0 ? p->cand_max_iter : 1;
  a.k = p->k;
  a.select_first = p->select_mode == BPSF_SELECT_FIRST;
  a.flags = p->flags;
  a.alpha = p->alpha;
  if (p->cand_mode == BPSF_TRIALS_TABLE) {
    a.n_trials = p->k > 0 ? (int)c->table_n : 0;
    a.trial_masks = c->table;
    a.mask_stride = c->table_stride;
    if (c->table64) a.flags |= SPARSE_FLAG_MASKS64;
  } else {
    a.n_trials = c->n_trials;
    a.trial_masks = static_cast<const uint32_t*>(c->masks.p);
    a.mask_stride = 0;
    // The empty trial (mask 0, the first of all subsets) decodes s itself
    // from fresh messages with the first BP's damping schedule: its run is
    // the first cand_max_iter iterations of the failed first BP, which never
    // reproduced s, so it cannot succeed. The kernels see the list from the
    // second mask on (trial indices shift by one, which keeps their order).
    if (empty_trial_skipped(p)) {
      a.trial_masks += 1;
      a.n_trials -= 1;
    }
  }
  // record: header, s bits per lane, every Phi column's share per lane, Phi
  const int kk = p->k > 0 ? p->k : 1;
  // (sparse family: header and Phi only)
  a.rec_stride = c->sparse >= 0 ? REC_HDR + kk : REC_HDR + G * (kk + 1) + kk;
  a.chunk = 2 * t.D;
  return 0;
}

// Scratch of a call carved out of a fixed region of `bytes` bytes at `base`
// (256-byte aligned): counters, then keys, then records.
struct FixedScratch {
  void* base = nullptr;
  size_t bytes = 0;
  bool keep = false;   // room past the records may hold kept trial corrections
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Largest buffer of kept trial corrections of a code (grown once per handle
// and kept).
constexpr size_t TRIAL_BITS_MAX = (size_t)256 << 20;

// The trials of a single-code call's first records (as many as
// TRIAL_BITS_MAX holds, one word per lane of a decode per trial) keep their
// corrections, so the re-run phase copies those winners' corrections instead
// of decoding up to cand_max_iter more iterations each: most of a small
// call's tail, and the whole re-run phase of a call whose failed shots fit.
// With a fixed scratch, only in the room it leaves past the records when the
// caller allows it (the request loop's single-code batches; not
// bpsf_decode_noalloc).
int keep_trial_bits(bpsf_code_s* c, const bpsf_params* p, int lanes, int64_t cap, const FixedScratch* fixed,
                    size_t fixed_used, Args* a)
{
  if (p->k <= 0 || (fixed && !fixed->keep)) return 0;
  const size_t per_rec = sizeof(uint32_t) * (size_t)(a->n_trials > 0 ? a->n_trials : 1) * (size_t)lanes;
  const size_t room = fixed ? (fixed->bytes > fixed_used ? fixed->bytes - fixed_used : 0) : TRIAL_BITS_MAX;
  const int64_t recs = std::min<int64_t>(cap, (int64_t)(room / per_rec));
  if (recs <= 0) return 0;
  if (fixed) {
    a->trial_bits = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(fixed->base) + fixed_used);
  } else {
    if (c->trial_bits.ensure(per_rec * (size_t)recs, TRIAL_BITS_MAX))
      return fail(BPSF_ENOMEM, "trial corrections of %lld records", (long long)recs);
    a->trial_bits = static_cast<uint32_t*>(c->trial_bits.p);
  }
  a->trial_bits_recs = recs;
  return 0;
}

int make_plan(bpsf_code_s* c, const bpsf_params* p, int64_t shots, Plan* pl, const FixedScratch* fixed = nullptr)
{
  const bool layered = (p->flags & BPSF_FLAG_LAYERED) != 0;
  if (layered && (c->wide >= 0 || c->sparse >= 0 || c->n_layers < 1))
    return fail(BPSF_ENOTSUP, "the layered schedule covers codes of the one-wave families with at most 254 layers");
  if (c->sparse >= 0 && p->precision != BPSF_PREC_FP32)
    return fail(BPSF_ENOTSUP, "codes of the sparse family decode with float messages only");
  if (p->k > 16 && c->sparse < 0) return fail(BPSF_ENOTSUP, "|Phi| above 16 needs a code of the sparse family");
  if (p->cand_mode == BPSF_TRIALS_TABLE && c->table64 && c->sparse < 0)
    return fail(BPSF_ENOTSUP, "64-bit trial lists need a code of the sparse family");
  if (p->k > 32 && !c->table64) return fail(BPSF_EINVAL, "|Phi| above 32 needs a 64-bit trial list");
  pl->wide = c->wide;
  pl->sparse = c->sparse;
  if (c->wide >= 0 || c->sparse >= 0) pl->tile = TileDesc{-1, 1};
  else if (pick_tile(c, &pl->tile, shots)) return fail(BPSF_ENOTSUP, "no kernel tile for this code");
  const TileDesc& t = pl->tile;
  Args& a = pl->args;
  int rc = fill_code_args(c, p, t, &a);
  if (rc) return rc;
  a.shots = shots;
  if (t.D > 0 && shots <= SMALL_CHUNK_SHOTS_PER_D * t.D) a.chunk = t.D;
  // scratch: one record and key per shot at most
  const int64_t cap = shots > 0 ? shots : 1;
  const size_t rec_bytes = sizeof(int32_t) * (size_t)a.rec_stride * (size_t)cap;
  const size_t key_bytes = sizeof(unsigned long long) * (size_t)cap;
  const size_t cnt_bytes = sizeof(unsigned long long) * CNT_WORDS;
  size_t fixed_used = 0;
  if (fixed) {
    const size_t need = align256(cnt_bytes) + align256(key_bytes) + rec_bytes;
    fixed_used = align256(need);
    if (need > fixed->bytes)
      return fail(BPSF_EINVAL, "%lld shots need %zu bytes of scratch; the fixed scratch holds %zu", (long long)shots,
                  need, fixed->bytes);
    unsigned char* b = static_cast<unsigned char*>(fixed->base);
    a.counters = reinterpret_cast<unsigned long long*>(b);
    a.keys = reinterpret_cast<unsigned long long*>(b + align256(cnt_bytes));
    a.records = reinterpret_cast<int32_t*>(b + align256(cnt_bytes) + align256(key_bytes));
  } else {
    if (c->records.ensure(rec_bytes) || c->keys.ensure(key_bytes) || c->counters.ensure(cnt_bytes))
      return fail(BPSF_ENOMEM, "scratch for %lld shots", (long long)shots);
    a.records = static_cast<int32_t*>(c->records.p);
    a.keys = static_cast<unsigned long long*>(c->keys.p);
    a.counters = static_cast<unsigned long long*>(c->counters.p);
  }
  a.rec_cap = cap;
  const bool fp64 = p->precision == BPSF_PREC_FP64;
  if (c->sparse >= 0) {
    const SparseDesc d = sparse_desc(c->sparse);
    if ((rc = keep_trial_bits(c, p, 64 * d.NW, cap, fixed, fixed_used, &a))) return rc;
    pl->lds = sparse_layout(c->sp_cells, c->M, d.NW, d.DVMAX, d.CPT).total;
    if (pl->lds > c->lds_max)
      return fail(BPSF_ENOTSUP, "the %d edges of this code need %zu bytes of LDS per workgroup, the device gives %zu",
                  c->E, pl->lds, c->lds_max);
    for (int mode = 0; mode < 3; ++mode) {
      int per_cu = 0;
      if (sparse_dispatch(1, c->sparse, mode, a, pl->lds, 0, nullptr, &per_cu) || per_cu < 1)
        return fail(BPSF_EDEVICE, "occupancy query failed for mode %d", mode);
      pl->grid[mode] = per_cu * c->cus;
    }
    return 0;
  }
  if (c->wide >= 0) {
    const WideDesc d = wide_desc(c->wide);
    pl->lds = wide_layout(fp64 ? 8 : 4, d.W, 64 * d.NW * d.IC, d.NW).total;
    if (pl->lds > c->lds_max)
      return fail(BPSF_ENOTSUP, "%s messages of this code need %zu bytes of LDS per workgroup, the device gives %zu",
                  fp64 ? "double" : "float", pl->lds, c->lds_max);
    for (int mode = 0; mode < 3; ++mode) {
      int per_cu = 0;
      if (wide_dispatch(1, c->wide, fp64, mode, a, pl->lds, 0, nullptr, &per_cu) || per_cu < 1)
        return fail(BPSF_EDEVICE, "occupancy query failed for mode %d", mode);
      pl->grid[mode] = per_cu * c->cus;
    }
    return 0;
  }
  if ((rc = keep_trial_bits(c, p, 64 / t.D, cap, fixed, fixed_used, &a))) return rc;
  pl->lds = tile_lds(c, t, fp64, c->uniform, layered);
  if (pl->lds > c->lds_max)
    return fail(BPSF_ENOTSUP, "this tile needs %zu bytes of LDS per workgroup, the device gives %zu", pl->lds,
                c->lds_max);
  for (int mode = 0; mode < 3; ++mode) {
    int per_cu = 0;
    if (occupancy(false, t, fp64, c->uniform, mode, pl->lds, &a, nullptr, &per_cu, layered))
      return fail(BPSF_EDEVICE, "occupancy query failed for mode %d", mode);
    if (c->tuned_wpc > 0 && c->tuned_wpc < per_cu) per_cu = c->tuned_wpc;
    pl->grid[mode] = per_cu * c->cus;
  }
  return 0;
}

}  // namespace

// Several codes decoded together (bpsf_mix_*): per-code task and record lists
// and a record pool shared by the codes.
struct bpsf_mix_s {
  int n = 0;
  bpsf_code_s* codes[MIX_MAX_CODES] = {};
  int fam = -1;
  DevBuf lists;      // [n][shots] int32 shot indices, grouped by code
  DevBuf rec_lists;  // [n][shots] int32 record indices of each code
  DevBuf records, keys;
  DevBuf counters;   // [n][CNT_WORDS] per code, then the mix words below
  DevBuf trial_bits; // kept corrections of converged trials, a region per code
  unsigned long long* last_counters = nullptr;   // counters of the last call (its scratch)
  std::mutex mu;
};

namespace {

// Mix words after the per-code counter blocks.
enum : int { MIX_TASKS = 0, MIX_REC_ALLOC = MIX_MAX_CODES, MIX_BAD = MIX_MAX_CODES + 1, MIX_WORDS = MIX_MAX_CODES + 2 };

// Checks a caller's CSR matrix and picks its kernel family, on the host
// alone: fills M, N, E, rw_max, cw_max, W, DV, wide and sparse of *c.
int classify_code(const int32_t* row_ptr, const int32_t* col_idx, int32_t M, int32_t N, bpsf_code_s* c)
{
  if (!row_ptr || M < 1 || N < 1) return fail(BPSF_EINVAL, "need M >= 1, N >= 1 and row_ptr");
  if (row_ptr[0] != 0) return fail(BPSF_EINVAL, "row_ptr[0] must be 0");
  for (int r = 0; r < M; ++r)
    if (row_ptr[r + 1] < row_ptr[r]) return fail(BPSF_EINVAL, "row_ptr must be non-decreasing");
  const int E = row_ptr[M];
  if (E > 0 && !col_idx) return fail(BPSF_EINVAL, "col_idx is NULL");
  std::vector<int> colw((size_t)N, 0);
  int rmin = 1 << 30, rmax = 0;
  for (int r = 0; r < M; ++r) {
    const int w = row_ptr[r + 1] - row_ptr[r];
    rmin = std::min(rmin, w);
    rmax = std::max(rmax, w);
    for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const int v = col_idx[e];
      if (v < 0 || v >= N) return fail(BPSF_EINVAL, "col_idx[%d] = %d out of range", e, v);
      if (e > row_ptr[r] && v <= col_idx[e - 1]) return fail(BPSF_EINVAL, "row %d: columns must ascend", r);
      ++colw[v];
    }
  }
  int cmin = 1 << 30, cmax = 0;
  for (int v = 0; v < N; ++v) {
    cmin = std::min(cmin, colw[v]);
    cmax = std::max(cmax, colw[v]);
  }
  if (M >= 65535) return fail(BPSF_ENOTSUP, "too many checks");
  if (rmin < 2) return fail(BPSF_ENOTSUP, "every check needs at least two bits");
  if (rmax > 255) return fail(BPSF_ENOTSUP, "rows heavier than 255");

  c->M = M;
  c->N = N;
  c->E = E;
  c->rw_max = rmax;
  c->cw_max = cmax;
  // a one-wave family when the code is regular and fits, else a wide one
  bool one_wave = false;
  if (rmin == rmax && cmin == cmax) {
    c->W = rmax;
    c->DV = cmax;
    TileDesc t;
    one_wave = pick_tile(c, &t) == 0;
  }
  if (!one_wave) {
    for (int f = 0; f < wide_count() && c->wide < 0; ++f) {
      const WideDesc d = wide_desc(f);
      const int G = 64 * d.NW;
      if (rmax <= d.W && cmax <= d.DV && M <= G * d.IC && N <= G * d.IV && (int64_t)N * d.DV <= 65535) {
        c->wide = f;
        c->W = d.W;
        c->DV = d.DV;
      }
    }
    for (int f = 0; f < sparse_count() && c->wide < 0 && c->sparse < 0; ++f) {
      const SparseDesc d = sparse_desc(f);
      const int T = 64 * d.NW;
      if (rmax <= d.WMAX && cmax <= d.DVMAX && M <= T * d.CPT && N <= T * d.BPT &&
          E + d.DVMAX + T * d.CPT <= 65535) {
        c->sparse = f;
        c->W = d.WMAX;
        c->DV = d.DVMAX;
      }
    }
    if (c->wide < 0 && c->sparse < 0)
      return fail(BPSF_ENOTSUP, "no kernel family for M=%d N=%d row weights %d..%d column weights %d..%d", M, N, rmin,
                  rmax, cmin, cmax);
  }
  return 0;
}

}  // namespace

extern "C" {

const char* bpsf_last_error(void) { return g_err.c_str(); }

int bpsf_load_code(const int32_t* row_ptr, const int32_t* col_idx, int32_t M, int32_t N, bpsf_code* out)
{
  if (!out) return fail(BPSF_EINVAL, "out is NULL");
  *out = nullptr;
  bpsf_code_s* c = new (std::nothrow) bpsf_code_s;
  if (!c) return fail(BPSF_ENOMEM, "handle");
  if (const int rc0 = classify_code(row_ptr, col_idx, M, N, c)) {
    delete c;
    return rc0;
  }
  const int E = c->E;
  // the sparse family's LDS layout, computed before any device work
  SparseTables sp;
  if (c->sparse >= 0) sparse_tables(row_ptr, col_idx, M, N, sparse_desc(c->sparse), &sp);
  const int W = c->W, DV = c->DV;

  // checks of every bit in ascending order (0xffff past its weight), the
  // bit's position in each row, the rows by position (-1 past the weight)
  std::vector<uint16_t> vchk((size_t)N * DV, 0xffff);
  std::vector<uint8_t> vpos((size_t)N * DV, 0);
  std::vector<int32_t> ell((size_t)M * W, -1);
  std::vector<uint8_t> roww((size_t)M);
  std::vector<int> fill((size_t)N, 0);
  for (int r = 0; r < M; ++r) {
    roww[r] = (uint8_t)(row_ptr[r + 1] - row_ptr[r]);
    for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const int v = col_idx[e];
      const int j = e - row_ptr[r];
      vchk[(size_t)v * DV + fill[v]] = (uint16_t)r;
      vpos[(size_t)v * DV + fill[v]] = (uint8_t)j;
      ++fill[v];
      ell[(size_t)r * W + j] = v;
    }
  }
  // layered schedule: in index order, every check takes the smallest layer
  // not held by an earlier check that shares a bit with it (one-wave codes)
  std::vector<uint8_t> layer;
  std::vector<uint16_t> ell16;
  if (c->wide < 0 && c->sparse < 0) {
    layer.assign((size_t)M, 0);
    std::vector<uint8_t> taken(256, 0);
    int nl = 0;
    for (int r = 0; r < M && nl <= 254; ++r) {
      std::fill(taken.begin(), taken.end(), 0);
      for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
        const int v = col_idx[e];
        for (int i = 0; i < DV; ++i) {
          const int r2 = vchk[(size_t)v * DV + i];
          if (r2 < r) taken[layer[(size_t)r2]] = 1;
        }
      }
      int l = 0;
      while (l < 255 && taken[(size_t)l]) ++l;
      layer[(size_t)r] = (uint8_t)l;
      nl = std::max(nl, l + 1);
    }
    c->n_layers = nl <= 254 ? nl : 0;
    ell16.resize(ell.size());
    for (size_t i = 0; i < ell.size(); ++i) ell16[i] = (uint16_t)ell[i];
  }
  int rc = 0;
  if (hipGetDevice(&c->device) != hipSuccess) rc = fail(BPSF_EDEVICE, "hipGetDevice");
  hipDeviceProp_t prop;
  if (!rc && hipGetDeviceProperties(&prop, c->device) != hipSuccess) rc = fail(BPSF_EDEVICE, "hipGetDeviceProperties");
  if (!rc) {
    c->cus = prop.multiProcessorCount;
    c->lds_max = prop.sharedMemPerBlock;
    // var_chk padded to whole 32-bit words: the kernels copy it by words
    if (c->var_chk.ensure((vchk.size() * 2 + 3) & ~(size_t)3) || c->var_pos.ensure(vpos.size()) ||
        c->ell_col.ensure(ell.size() * 4) || c->row_w.ensure(roww.size()))
      rc = fail(BPSF_ENOMEM, "code tables");
  }
  if (!rc && (hipMemcpy(c->var_chk.p, vchk.data(), vchk.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(c->var_pos.p, vpos.data(), vpos.size(), hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(c->ell_col.p, ell.data(), ell.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(c->row_w.p, roww.data(), roww.size(), hipMemcpyHostToDevice) != hipSuccess))
    rc = fail(BPSF_EDEVICE, "uploading code tables");
  if (!rc && c->sparse >= 0) {
    const SparseTables& t = sp;
    c->sp_cells = t.cells;
    if (c->sp_roff.ensure(t.roff.size() * 2) || c->sp_echk.ensure(t.echk.size() * 2) ||
        c->sp_bits.ensure(t.bits.size() * 4) || c->sp_rw.ensure(t.rw.size()) || c->sp_rperm.ensure(t.rperm.size() * 2) ||
        c->sp_cperm.ensure(t.cperm.size() * 2) || c->sp_cinv.ensure(t.cinv.size() * 2))
      rc = fail(BPSF_ENOMEM, "sparse tables");
    else if (hipMemcpy(c->sp_roff.p, t.roff.data(), t.roff.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->sp_echk.p, t.echk.data(), t.echk.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->sp_bits.p, t.bits.data(), t.bits.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->sp_rw.p, t.rw.data(), t.rw.size(), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->sp_rperm.p, t.rperm.data(), t.rperm.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->sp_cperm.p, t.cperm.data(), t.cperm.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->sp_cinv.p, t.cinv.data(), t.cinv.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
      rc = fail(BPSF_EDEVICE, "uploading sparse tables");
  }
  if (!rc && c->wide < 0 && c->sparse < 0) {
    if (c->check_layer.ensure(layer.size()) || c->ell16.ensure(ell16.size() * 2))
      rc = fail(BPSF_ENOMEM, "layer tables");
    else if (hipMemcpy(c->check_layer.p, layer.data(), layer.size(), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(c->ell16.p, ell16.data(), ell16.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
      rc = fail(BPSF_EDEVICE, "uploading layer tables");
  }
  // per-call tables at their largest size now, so that no decode call has
  // to allocate them: channel LLRs, the initial messages of a wide code, the
  // largest generated trial list (2^16 masks)
  if (!rc && (c->llr64.ensure(sizeof(double) * (size_t)N) || c->llr32.ensure(sizeof(float) * (size_t)N) ||
              c->masks.ensure(sizeof(uint32_t) * ((size_t)1 << 16))))
    rc = fail(BPSF_ENOMEM, "LLR and trial tables");
  if (!rc && c->wide >= 0) {
    const WideDesc d = wide_desc(c->wide);
    const size_t n = (size_t)c->W * 64 * d.NW * d.IC;
    if (c->init64.ensure(sizeof(double) * n) || c->init32.ensure(sizeof(float) * n))
      rc = fail(BPSF_ENOMEM, "initial message tables");
  }
  if (rc) { delete c; return rc; }
  if (c->wide >= 0) c->ell_host = std::move(ell);
  *out = c;
  return 0;
}

void bpsf_free_code(bpsf_code code)
{
  if (!code) return;
  (void)hipDeviceSynchronize();
  delete code;
}

int bpsf_code_info(bpsf_code c, int32_t* M, int32_t* N, int32_t* edges, int32_t* rw, int32_t* cw)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  if (M) *M = c->M;
  if (N) *N = c->N;
  if (edges) *edges = c->E;
  if (rw) *rw = c->rw_max;
  if (cw) *cw = c->cw_max;
  return 0;
}

int bpsf_sparse_layout(const int32_t* row_ptr, const int32_t* col_idx, int32_t M, int32_t N, int32_t* info,
                       uint16_t* roff, uint8_t* rw, uint32_t* bits, uint16_t* cperm, uint16_t* rperm)
{
  if (!info) return fail(BPSF_EINVAL, "info is NULL");
  bpsf_code_s c;
  if (const int rc = classify_code(row_ptr, col_idx, M, N, &c)) return rc;
  for (int i = 0; i < BPSF_SPARSE_INFO_WORDS; ++i) info[i] = 0;
  info[0] = c.sparse;
  if (c.sparse < 0) return 0;
  const SparseDesc d = sparse_desc(c.sparse);
  SparseTables t;
  sparse_tables(row_ptr, col_idx, M, N, d, &t);
  info[1] = t.cells;
  info[2] = d.WMAX;
  info[3] = 64 * d.NW;
  info[4] = d.CPT;
  info[5] = d.DVMAX;
  info[6] = t.overflow;
  info[7] = t.extra_positions;
  info[8] = t.folded;
  if (roff) std::copy(t.roff.begin(), t.roff.end(), roff);
  if (rw) std::copy(t.rw.begin(), t.rw.end(), rw);
  if (bits) std::copy(t.bits.begin(), t.bits.end(), bits);
  if (cperm) std::copy(t.cperm.begin(), t.cperm.end(), cperm);
  if (rperm) std::copy(t.rperm.begin(), t.rperm.end(), rperm);
  return 0;
}

}  // extern "C"

namespace {

// One decode call: the three phases of Algorithm 1 as stream-ordered launches,
// with the handle's scratch (fixed == NULL) or a fixed region.
int decode_call(bpsf_code c, const uint8_t* syndromes, const double* priors, int64_t shots, const bpsf_params* p,
                uint8_t* corrections, uint8_t* converged, int32_t* iterations, void* stream,
                const FixedScratch* fixed)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (shots < 0) return fail(BPSF_EINVAL, "shots < 0");
  if (shots > 0x7fffffffLL) return fail(BPSF_EINVAL, "at most 2^31-1 shots per call");
  if (shots > 0 && (!syndromes || !corrections || !converged || !iterations))
    return fail(BPSF_EINVAL, "NULL buffer");
  std::lock_guard<std::mutex> lk(c->mu);
  if ((rc = update_llr(c, priors, stream))) return rc;
  if (shots == 0) return 0;
  if ((rc = update_masks(c, p, stream))) return rc;
  Plan pl;
  if ((rc = make_plan(c, p, shots, &pl, fixed))) return rc;
  Args& a = pl.args;
  a.syndromes = syndromes;
  a.corrections = corrections;
  a.converged = converged;
  a.iterations = iterations;
  const bool fp64 = p->precision == BPSF_PREC_FP64;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  c->last_counters = a.counters;
  if (reset_counters(a.counters, CNT_WORDS, stream)) return fail(BPSF_EDEVICE, "counter reset launch");
  auto launch = [&](int mode) {
    // no more workgroups than the phase can have tasks (one decode per
    // workgroup) or chunks of tasks (one-wave kernels): every shot (a first
    // BP or a re-run) or every trial of every shot
    const long long most = mode == MODE_CAND ? shots * (long long)a.n_trials : shots;
    const int groups = most < pl.grid[mode] ? (int)std::max(1LL, most) : pl.grid[mode];
    if (pl.sparse >= 0) return sparse_dispatch(0, pl.sparse, mode, a, pl.lds, groups, stream, nullptr);
    if (pl.wide >= 0) return wide_dispatch(0, pl.wide, fp64, mode, a, pl.lds, groups, stream, nullptr);
    const long long chunks = (most + a.chunk - 1) / a.chunk;
    const int grid = chunks < pl.grid[mode] ? (int)std::max(1LL, chunks) : pl.grid[mode];
    return tile_dispatch(0, pl.tile, fp64, c->uniform, mode, false, a, pl.lds, grid, stream, nullptr,
                         (p->flags & BPSF_FLAG_LAYERED) != 0);
  };
  if (c->timing) HIP_OK(hipEventRecord(c->ev[0], st));
  if (launch(MODE_MAIN)) return fail(BPSF_EDEVICE, "first-BP launch failed");
  if (c->timing) HIP_OK(hipEventRecord(c->ev[1], st));
  if (p->k > 0) {
    if (launch(MODE_CAND)) return fail(BPSF_EDEVICE, "trial launch failed");
    if (c->timing) HIP_OK(hipEventRecord(c->ev[2], st));
    if (launch(MODE_EMIT)) return fail(BPSF_EDEVICE, "re-run launch failed");
    if (c->timing) HIP_OK(hipEventRecord(c->ev[3], st));
  }
  c->timed_last = c->timing;
  c->timed_phases = p->k > 0 ? 3 : 1;
  return 0;
}

// The fixed scratch of bpsf_decode_noalloc: one copy per device, held until
// the process ends. Host code never uses the array's name as an address: it
// asks the runtime for each device's copy once (with that device current)
// and passes that address to the kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;   // device -> its copy of `scratch`

int scratch_address(int dev, void** out)
{
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return 0;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(BPSF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch_addr[dev] = ptr;
  *out = ptr;
  return 0;
}

}  // namespace

extern "C" {

int bpsf_decode(bpsf_code c, const uint8_t* syndromes, const double* priors, int64_t shots,
                const bpsf_params* p, uint8_t* corrections, uint8_t* converged, int32_t* iterations,
                void* stream)
{
  return decode_call(c, syndromes, priors, shots, p, corrections, converged, iterations, stream, nullptr);
}

int bpsf_decode_noalloc(bpsf_code c, const uint8_t* syndromes, const double* priors, int64_t shots,
                        const bpsf_params* p, uint8_t* corrections, uint8_t* converged, int32_t* iterations,
                        void* stream)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BPSF_EDEVICE, "hipGetDevice");
  if (dev != c->device)
    return fail(BPSF_EINVAL, "the current device (%d) is not the code's device (%d)", dev, c->device);
  FixedScratch fx;
  int rc = scratch_address(dev, &fx.base);
  if (rc) return rc;
  fx.bytes = NOALLOC_SCRATCH_BYTES;
  return decode_call(c, syndromes, priors, shots, p, corrections, converged, iterations, stream, &fx);
}

int bpsf_set_timing(bpsf_code c, int enable)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  if (enable && !c->ev[0])
    for (auto& e : c->ev) HIP_OK(hipEventCreate(&e));
  c->timing = enable != 0;
  return 0;
}

int bpsf_last_timing(bpsf_code c, float* ms)
{
  if (!c || !ms) return fail(BPSF_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  for (int i = 0; i < 4; ++i) ms[i] = 0.f;
  if (!c->timed_last) return fail(BPSF_EINVAL, "the last decode on this handle was not timed");
  const int last = c->timed_phases;
  HIP_OK(hipEventSynchronize(c->ev[last]));
  HIP_OK(hipEventElapsedTime(&ms[0], c->ev[0], c->ev[last]));
  for (int i = 0; i < last; ++i) HIP_OK(hipEventElapsedTime(&ms[i + 1], c->ev[i], c->ev[i + 1]));
  return 0;
}

int bpsf_last_stats(bpsf_code c, void* stream, bpsf_stats* out)
{
  if (!c || !out) return fail(BPSF_EINVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  if (!c->last_counters) return 0;
  unsigned long long h[CNT_WORDS];
  HIP_OK(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  HIP_OK(hipMemcpy(h, c->last_counters, sizeof h, hipMemcpyDeviceToHost));
  out->main_iterations = (int64_t)h[ST_MAIN_ITERS];
  out->trial_iterations = (int64_t)h[ST_CAND_ITERS];
  out->rerun_iterations = (int64_t)h[ST_EMIT_ITERS];
  out->failed_shots = (int64_t)h[CNT_FAILED];
  out->converged_trials = (int64_t)h[ST_CAND_CONV];
  out->errors = (int64_t)h[ST_ERRORS];
  return 0;
}

int64_t bpsf_num_trials(const bpsf_params* p, uint32_t* masks_out, int64_t cap)
{
  int rc = check_params(p);
  if (rc) return rc;
  if (p->cand_mode == BPSF_TRIALS_TABLE) return fail(BPSF_EINVAL, "a BPSF_TRIALS_TABLE list is the caller's");
  const std::vector<uint32_t> m = trial_masks(p->k, p->cand_mode, p->w_max);
  if (masks_out)
    for (int64_t i = 0; i < (int64_t)m.size() && i < cap; ++i) masks_out[i] = m[(size_t)i];
  return (int64_t)m.size();
}

int bpsf_bp_trace(bpsf_code c, const uint8_t* syndrome, const double* priors, const bpsf_params* p,
                  void* lout_trace, void* c2v_trace, uint8_t* hard_out, int32_t* iters_out, uint8_t* conv_out)
{
  if (!c || !syndrome || !hard_out || !iters_out || !conv_out) return fail(BPSF_EINVAL, "NULL argument");
  int rc = check_params(p);
  if (rc) return rc;
  if (c->wide >= 0 || c->sparse >= 0)
    return fail(BPSF_ENOTSUP, "per-iteration traces cover codes of the one-wave families");
  bpsf_params q = *p;
  q.k = 0;
  std::lock_guard<std::mutex> lk(c->mu);
  if ((rc = update_llr(c, priors, nullptr))) return rc;
  Plan pl;
  if ((rc = make_plan(c, &q, 1, &pl))) return rc;
  const size_t rb = q.precision == BPSF_PREC_FP64 ? 8 : 4;
  const size_t nl = rb * (size_t)q.max_iter * (size_t)c->N;
  const size_t nc = rb * (size_t)q.max_iter * (size_t)c->M * (size_t)c->W;
  DevBuf dsyn, dcorr, dconv, dit, dl, dc;
  if (dsyn.ensure(c->M) || dcorr.ensure(c->N) || dconv.ensure(1) || dit.ensure(4) || dl.ensure(nl) || dc.ensure(nc))
    return fail(BPSF_ENOMEM, "trace buffers");
  HIP_OK(hipMemcpy(dsyn.p, syndrome, c->M, hipMemcpyHostToDevice));
  HIP_OK(hipMemset(dl.p, 0, nl));
  HIP_OK(hipMemset(dc.p, 0, nc));
  Args& a = pl.args;
  a.syndromes = static_cast<const uint8_t*>(dsyn.p);
  a.corrections = static_cast<uint8_t*>(dcorr.p);
  a.converged = static_cast<uint8_t*>(dconv.p);
  a.iterations = static_cast<int32_t*>(dit.p);
  a.trace_lout = dl.p;
  a.trace_c2v = dc.p;
  if (reset_counters(a.counters, CNT_WORDS, nullptr)) return fail(BPSF_EDEVICE, "counter reset launch");
  if (tile_dispatch(0, pl.tile, q.precision == BPSF_PREC_FP64, c->uniform, MODE_MAIN, true, a, pl.lds, 1, nullptr, nullptr,
                    (q.flags & BPSF_FLAG_LAYERED) != 0))
    return fail(BPSF_EDEVICE, "trace launch failed");
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(hard_out, dcorr.p, c->N, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(conv_out, dconv.p, 1, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(iters_out, dit.p, 4, hipMemcpyDeviceToHost));
  if (lout_trace) HIP_OK(hipMemcpy(lout_trace, dl.p, nl, hipMemcpyDeviceToHost));
  if (c2v_trace) HIP_OK(hipMemcpy(c2v_trace, dc.p, nc, hipMemcpyDeviceToHost));
  return 0;
}

int bpsf_mix_create(const bpsf_code* codes, int32_t n_codes, bpsf_mix* out)
{
  if (!out) return fail(BPSF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!codes || n_codes < 1 || n_codes > MIX_MAX_CODES)
    return fail(BPSF_EINVAL, "need 1..%d codes", MIX_MAX_CODES);
  int fam = -1;
  for (int i = 0; i < n_codes; ++i) {
    if (!codes[i]) return fail(BPSF_EINVAL, "codes[%d] is NULL", i);
    for (int j = 0; j < i; ++j)
      if (codes[j] == codes[i]) return fail(BPSF_EINVAL, "codes[%d] repeats codes[%d]", i, j);
    if (codes[i]->device != codes[0]->device) return fail(BPSF_EINVAL, "codes live on different devices");
    TileDesc t;
    if (pick_tile(codes[i], &t)) return fail(BPSF_ENOTSUP, "codes[%d] has no kernel tile", i);
    if (fam >= 0 && t.fam != fam)
      return fail(BPSF_ENOTSUP, "codes[%d] needs another kernel family than codes[0]", i);
    fam = t.fam;
  }
  bpsf_mix_s* m = new (std::nothrow) bpsf_mix_s;
  if (!m) return fail(BPSF_ENOMEM, "handle");
  m->n = n_codes;
  for (int i = 0; i < n_codes; ++i) m->codes[i] = codes[i];
  m->fam = fam;
  *out = m;
  return 0;
}

void bpsf_mix_free(bpsf_mix m)
{
  if (!m) return;
  (void)hipDeviceSynchronize();
  delete m;
}

}  // extern "C"

namespace {

// Shots of the mix either listed by code index (shot_code, device) or
// grouped: code c's shots are the counts[c] rows after those of codes < c.
// Record words per shot that cover every tile a mixed call of up to `shots`
// shots can take (the mixed tile, and the tiles of small or single-code calls).
int mix_stride_max(bpsf_mix m, int64_t shots, const bpsf_params* p, int* out)
{
  int stride = 0, rc = 0;
  for (int i = 0; i < m->n; ++i) {
    for (int64_t call : {(int64_t)-1, std::min(shots, SMALL_CALL_SHOTS_PER_D), std::min(shots, SMALL_CALL_SHOTS)}) {
      TileDesc t;
      Args a;
      if (pick_tile(m->codes[i], &t, call)) return fail(BPSF_ENOTSUP, "code %d has no kernel tile", i);
      if ((rc = fill_code_args(m->codes[i], p, t, &a))) return rc;
      stride = std::max(stride, a.rec_stride);
    }
  }
  *out = stride;
  return 0;
}

// Scratch of a grouped mixed call in a fixed region: counters, keys, the
// per-code record lists, then the records.
size_t mix_fixed_bytes(int n_codes, int64_t shots, int stride)
{
  const size_t n = (size_t)shots;
  return align256(sizeof(unsigned long long) * ((size_t)CNT_WORDS * n_codes + MIX_WORDS)) +
         align256(sizeof(unsigned long long) * n) + align256(sizeof(int32_t) * n * (size_t)n_codes) +
         sizeof(int32_t) * n * (size_t)stride;
}

int mix_decode(bpsf_mix m, const int32_t* shot_code, const int64_t* counts, const uint8_t* syndromes,
               int64_t syn_stride, const double* const* priors, int64_t shots, const bpsf_params* p,
               uint8_t* corrections, int64_t corr_stride, uint8_t* converged, int32_t* iterations, void* stream,
               const FixedScratch* fixed = nullptr)
{
  if (!m) return fail(BPSF_EINVAL, "mix is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (p->flags & BPSF_FLAG_LAYERED) return fail(BPSF_ENOTSUP, "mixed-code calls run the flooding schedule only");
  if (p->k > 16) return fail(BPSF_ENOTSUP, "mixed-code calls take |Phi| up to 16");
  if (p->cand_mode == BPSF_TRIALS_TABLE)
    for (int i = 0; i < m->n; ++i)
      if (m->codes[i]->table64) return fail(BPSF_ENOTSUP, "mixed-code calls take 32-bit trial lists only");
  if (shots < 0) return fail(BPSF_EINVAL, "shots < 0");
  if (shots > 0x7fffffffLL) return fail(BPSF_EINVAL, "at most 2^31-1 shots per call");
  if (!priors) return fail(BPSF_EINVAL, "priors is NULL");
  for (int i = 0; i < m->n; ++i) {
    if (syn_stride < m->codes[i]->M) return fail(BPSF_EINVAL, "syn_stride %lld < M = %d of code %d", (long long)syn_stride, m->codes[i]->M, i);
    if (corr_stride < m->codes[i]->N) return fail(BPSF_EINVAL, "corr_stride %lld < N = %d of code %d", (long long)corr_stride, m->codes[i]->N, i);
  }
  if (shots > 0 && ((!shot_code && !counts) || !syndromes || !corrections || !converged || !iterations))
    return fail(BPSF_EINVAL, "NULL buffer");
  std::lock_guard<std::mutex> lk(m->mu);
  // the codes' LLR and trial tables (each code's own lock; a fixed order)
  bool uniform = true;
  for (int i = 0; i < m->n; ++i) {
    bpsf_code_s* c = m->codes[i];
    std::lock_guard<std::mutex> lc(c->mu);
    if ((rc = update_llr(c, priors[i], stream))) return rc;
    if ((rc = update_masks(c, p, stream))) return rc;
    uniform = uniform && c->uniform;
  }
  if (shots == 0) return 0;
  const bool fp64 = p->precision == BPSF_PREC_FP64;
  MixArgs ma;
  memset(&ma, 0, sizeof ma);
  ma.n_codes = m->n;
  size_t lds = 0;
  int stride = 0;
  // grouped shots of a single code run that code's own kernels (the same
  // decode body, arguments in registers), with the tile a single-code call of
  // as many shots would take
  int only = -1;
  if (counts)
    for (int i = 0; i < m->n; ++i)
      if (counts[i] > 0) only = only == -1 ? i : -2;
  // a small mixed call runs the tiles single-code calls of its size would
  // take when they share a family (the small family, for codes it fits)
  int fam = m->fam;
  bool small = only < 0 && shots <= SMALL_CALL_SHOTS;
  for (int i = 0, f0 = -1; i < m->n && small; ++i) {
    TileDesc t;
    if (pick_tile(m->codes[i], &t, shots, SMALL_MIX_SHOTS_PER_D) || (f0 >= 0 && t.fam != f0)) {
      small = false;
    } else {
      f0 = t.fam;
      fam = t.fam;
    }
  }
  if (!small) fam = m->fam;
  TileDesc tiles[MIX_MAX_CODES];
  for (int i = 0; i < m->n; ++i) {
    bpsf_code_s* c = m->codes[i];
    if (i == only) {
      if (pick_tile(c, &tiles[i], counts[i])) return fail(BPSF_ENOTSUP, "code %d has no kernel tile", i);
    } else if (small) {
      if (pick_tile(c, &tiles[i], shots, SMALL_MIX_SHOTS_PER_D)) return fail(BPSF_ENOTSUP, "code %d has no kernel tile", i);
    } else if (pick_tile(c, &tiles[i]) || tiles[i].fam != m->fam) {
      return fail(BPSF_ENOTSUP, "code %d changed kernel family", i);
    }
    if ((rc = fill_code_args(c, p, tiles[i], &ma.code[i]))) return rc;
    if ((i == only ? counts[i] : shots) <= SMALL_CHUNK_SHOTS_PER_D * tiles[i].D) ma.code[i].chunk = tiles[i].D;
    // a mixed launch runs the uniform-LLR kernel only when every code qualifies
    lds = std::max(lds, tile_lds(c, tiles[i], fp64, uniform));
    stride = std::max(stride, ma.code[i].rec_stride);
    ma.cost[i] = 1.0f / (float)tiles[i].D;   // a wave iteration costs the same for every D
  }
  // scratch
  const size_t n = (size_t)shots;
  const size_t words = (size_t)CNT_WORDS * m->n + MIX_WORDS;
  void *lists = nullptr, *rec_lists = nullptr, *records = nullptr, *keys = nullptr, *counters = nullptr;
  if (fixed) {
    // grouped calls only (no shot lists)
    const size_t need = mix_fixed_bytes(m->n, shots, stride);
    if (counts == nullptr || need > fixed->bytes)
      return fail(BPSF_EINVAL, "%lld shots need %zu bytes of scratch; the region holds %zu", (long long)shots, need,
                  fixed->bytes);
    unsigned char* b = static_cast<unsigned char*>(fixed->base);
    counters = b;
    b += align256(sizeof(unsigned long long) * words);
    keys = b;
    b += align256(sizeof(unsigned long long) * n);
    rec_lists = b;
    b += align256(sizeof(int32_t) * n * (size_t)m->n);
    records = b;
  } else {
    if ((!counts && m->lists.ensure(sizeof(int32_t) * n * m->n)) || m->rec_lists.ensure(sizeof(int32_t) * n * m->n) ||
        m->records.ensure(sizeof(int32_t) * n * (size_t)stride) || m->keys.ensure(sizeof(unsigned long long) * n) ||
        m->counters.ensure(sizeof(unsigned long long) * words))
      return fail(BPSF_ENOMEM, "scratch for %lld shots", (long long)shots);
    lists = m->lists.p;
    rec_lists = m->rec_lists.p;
    records = m->records.p;
    keys = m->keys.p;
    counters = m->counters.p;
  }
  unsigned long long* cnt = static_cast<unsigned long long*>(counters);
  unsigned long long* mixw = cnt + (size_t)CNT_WORDS * m->n;
  m->last_counters = cnt;
  int64_t base = 0;
  for (int i = 0; i < m->n; ++i) {
    Args& a = ma.code[i];
    a.syndromes = syndromes;
    a.syn_stride = syn_stride;
    a.shots = shots;
    a.corrections = corrections;
    a.corr_stride = corr_stride;
    a.converged = converged;
    a.iterations = iterations;
    if (counts) {
      a.shots = counts[i];
      a.shot_base = base;
      base += counts[i];
    } else {
      a.task_shot = static_cast<const int32_t*>(lists) + (size_t)i * n;
      a.task_count = mixw + MIX_TASKS + i;
    }
    a.rec_list = static_cast<int32_t*>(rec_lists) + (size_t)i * n;
    a.rec_alloc = mixw + MIX_REC_ALLOC;
    a.records = static_cast<int32_t*>(records);
    a.rec_stride = stride;
    a.rec_cap = shots;
    a.keys = static_cast<unsigned long long*>(keys);
    a.counters = cnt + (size_t)CNT_WORDS * i;
  }
  // kept trial corrections (calls of the mixed kernel's small form, and
  // grouped calls of one code): the codes share the record numbers, and each
  // code's decodes have lanes of their own, so every code keeps the same
  // first records in a region of its own (with a fixed scratch, in the room
  // past the call's when the caller allows it)
  const bool small_form = shots <= SMALL_CALL_SHOTS;
  if (p->k > 0 && (!fixed || fixed->keep) && (small_form || only >= 0)) {
    size_t per_rec[MIX_MAX_CODES] = {}, sum = 0;
    for (int i = 0; i < m->n; ++i)
      if (!counts || counts[i] > 0) {
        const Args& a = ma.code[i];
        per_rec[i] = sizeof(uint32_t) * (size_t)(a.n_trials > 0 ? a.n_trials : 1) * (size_t)(64 / tiles[i].D);
        sum += per_rec[i];
      }
    const size_t used = fixed ? align256(mix_fixed_bytes(m->n, shots, stride)) : 0;
    const size_t room = fixed ? (fixed->bytes > used ? fixed->bytes - used : 0) : TRIAL_BITS_MAX;
    const int64_t recs = sum ? std::min<int64_t>(shots, (int64_t)(room / sum)) : 0;
    if (recs > 0) {
      unsigned char* kb = nullptr;
      if (fixed) {
        kb = static_cast<unsigned char*>(fixed->base) + used;
      } else {
        if (m->trial_bits.ensure(sum * (size_t)recs, TRIAL_BITS_MAX))
          return fail(BPSF_ENOMEM, "trial corrections of %lld records", (long long)recs);
        kb = static_cast<unsigned char*>(m->trial_bits.p);
      }
      for (int i = 0; i < m->n; ++i) {
        if (!per_rec[i]) continue;
        ma.code[i].trial_bits = reinterpret_cast<uint32_t*>(kb);
        ma.code[i].trial_bits_recs = recs;
        kb += per_rec[i] * (size_t)recs;
      }
    }
  }
  BucketArgs b;
  memset(&b, 0, sizeof b);
  b.shot_code = shot_code;
  b.shots = shots;
  b.n_codes = m->n;
  b.lists = static_cast<int32_t*>(lists);
  for (int i = 0; i < m->n; ++i) b.counts[i] = mixw + MIX_TASKS + i;
  b.bad = mixw + MIX_BAD;
  if (only >= 0) {
    bpsf_code_s* c = m->codes[only];
    const Args& a = ma.code[only];
    const size_t l1 = tile_lds(c, tiles[only], fp64, c->uniform);
    if (reset_counters(cnt, (int)words, stream)) return fail(BPSF_EDEVICE, "counter reset launch");
    for (int mode = 0; mode < (p->k > 0 ? 3 : 1); ++mode) {
      int per_cu = 0;
      if (occupancy(false, tiles[only], fp64, c->uniform, mode, l1, &a, nullptr, &per_cu))
        return fail(BPSF_EDEVICE, "occupancy query failed for mode %d", mode);
      // no more waves than the phase can have chunks of tasks
      const long long most = mode == MODE_CAND ? a.shots * (long long)a.n_trials : a.shots;
      const long long chunks = (most + a.chunk - 1) / a.chunk;
      const int grid = chunks < per_cu * c->cus ? (int)std::max(1LL, chunks) : per_cu * c->cus;
      if (tile_dispatch(0, tiles[only], fp64, c->uniform, mode, false, a, l1, grid, stream, nullptr))
        return fail(BPSF_EDEVICE, "launch of phase %d failed", mode);
    }
    return 0;
  }
  int grid[3];
  for (int mode = 0; mode < 3; ++mode) {
    int per_cu = 0;
    if (occupancy(true, TileDesc{fam, 0}, fp64, uniform, mode, lds, nullptr, &ma, &per_cu, false, small_form))
      return fail(BPSF_EDEVICE, "occupancy query failed for mode %d", mode);
    grid[mode] = per_cu * m->codes[0]->cus;
  }
  if (reset_counters(cnt, (int)words, stream)) return fail(BPSF_EDEVICE, "counter reset launch");
  if (!counts && bucket_launch(b, stream)) return fail(BPSF_EDEVICE, "bucketing launch failed");
  if (mixed_dispatch(0, fam, fp64, uniform, small_form, MODE_MAIN, ma, lds, grid[MODE_MAIN], stream, nullptr))
    return fail(BPSF_EDEVICE, "first-BP launch failed");
  if (p->k > 0) {
    if (mixed_dispatch(0, fam, fp64, uniform, small_form, MODE_CAND, ma, lds, grid[MODE_CAND], stream, nullptr))
      return fail(BPSF_EDEVICE, "trial launch failed");
    if (mixed_dispatch(0, fam, fp64, uniform, small_form, MODE_EMIT, ma, lds, grid[MODE_EMIT], stream, nullptr))
      return fail(BPSF_EDEVICE, "re-run launch failed");
  }
  return 0;
}

}  // namespace

extern "C" {

int bpsf_mix_decode(bpsf_mix m, const int32_t* shot_code, const uint8_t* syndromes, int64_t syn_stride,
                    const double* const* priors, int64_t shots, const bpsf_params* p, uint8_t* corrections,
                    int64_t corr_stride, uint8_t* converged, int32_t* iterations, void* stream)
{
  return mix_decode(m, shot_code, nullptr, syndromes, syn_stride, priors, shots, p, corrections, corr_stride,
                    converged, iterations, stream);
}

int bpsf_mix_decode_grouped(bpsf_mix m, const int64_t* counts, const uint8_t* syndromes, int64_t syn_stride,
                            const double* const* priors, const bpsf_params* p, uint8_t* corrections,
                            int64_t corr_stride, uint8_t* converged, int32_t* iterations, void* stream)
{
  if (!m || !counts) return fail(BPSF_EINVAL, "NULL argument");
  int64_t shots = 0;
  for (int i = 0; i < m->n; ++i) {
    if (counts[i] < 0) return fail(BPSF_EINVAL, "counts[%d] < 0", i);
    shots += counts[i];
  }
  return mix_decode(m, nullptr, counts, syndromes, syn_stride, priors, shots, p, corrections, corr_stride,
                    converged, iterations, stream);
}

int bpsf_mix_last_stats(bpsf_mix m, void* stream, bpsf_stats* per_code, int64_t* invalid_shots)
{
  if (!m || !per_code) return fail(BPSF_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(m->mu);
  for (int i = 0; i < m->n; ++i) memset(&per_code[i], 0, sizeof per_code[i]);
  if (invalid_shots) *invalid_shots = 0;
  if (!m->last_counters) return 0;
  std::vector<unsigned long long> h((size_t)CNT_WORDS * m->n + MIX_WORDS);
  HIP_OK(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  HIP_OK(hipMemcpy(h.data(), m->last_counters, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
  for (int i = 0; i < m->n; ++i) {
    const unsigned long long* w = h.data() + (size_t)CNT_WORDS * i;
    per_code[i].main_iterations = (int64_t)w[ST_MAIN_ITERS];
    per_code[i].trial_iterations = (int64_t)w[ST_CAND_ITERS];
    per_code[i].rerun_iterations = (int64_t)w[ST_EMIT_ITERS];
    per_code[i].failed_shots = (int64_t)w[CNT_FAILED];
    per_code[i].converged_trials = (int64_t)w[ST_CAND_CONV];
    per_code[i].errors = (int64_t)w[ST_ERRORS];
  }
  if (invalid_shots) *invalid_shots = (int64_t)h[(size_t)CNT_WORDS * m->n + MIX_BAD];
  return 0;
}

int bpsf_tile_options(bpsf_code c, int32_t* d_out, int32_t cap)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  int n = 0;
  for (int D = MAX_D; D >= 1; D >>= 1) {
    bool fits = false;
    for (int fam = 0; fam < family_count() && !fits; ++fam) fits = tile_fits(c, fam, D);
    if (fits) {
      if (d_out && n < cap) d_out[n] = D;
      ++n;
    }
  }
  return n;
}

int bpsf_set_tile(bpsf_code c, int32_t decodes_per_wave, int32_t waves_per_cu)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  if (waves_per_cu < 0) return fail(BPSF_EINVAL, "waves_per_cu < 0");
  bool ok = decodes_per_wave == 0;
  for (int fam = 0; fam < family_count() && !ok; ++fam) ok = tile_fits(c, fam, decodes_per_wave);
  if (!ok) return fail(BPSF_EINVAL, "the code does not fit %d decodes per wave", decodes_per_wave);
  std::lock_guard<std::mutex> lk(c->mu);
  c->tuned_D = decodes_per_wave;
  c->tuned_wpc = waves_per_cu;
  return 0;
}

int bpsf_autotune(bpsf_code c, const uint8_t* syndromes, const double* priors, int64_t shots,
                  const bpsf_params* p, int32_t reps, void* stream, bpsf_tuning* out)
{
  if (!c || !out) return fail(BPSF_EINVAL, "NULL argument");
  if (c->wide >= 0 || c->sparse >= 0) return fail(BPSF_ENOTSUP, "the launch shape of a wide or sparse code is fixed");
  if (shots < 1 || !syndromes) return fail(BPSF_EINVAL, "need a sample of at least one shot");
  if (reps < 1) return fail(BPSF_EINVAL, "reps < 1");
  int rc = check_params(p);
  if (rc) return rc;
  memset(out, 0, sizeof *out);
  DevBuf corr, conv, it;
  if (corr.ensure((size_t)shots * c->N) || conv.ensure((size_t)shots) || it.ensure(sizeof(int32_t) * (size_t)shots))
    return fail(BPSF_ENOMEM, "autotune outputs");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  int32_t ds[8];
  const int nd = bpsf_tile_options(c, ds, 8);
  const int saved_D = c->tuned_D, saved_w = c->tuned_wpc;
  float best = 0.f;
  int best_D = 0, best_w = 0, tried = 0;
  rc = 0;
  for (int i = 0; i < nd && !rc; ++i) {
    // resident waves per CU this tile allows
    int max_w = 0;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->tuned_D = ds[i];
      c->tuned_wpc = 0;
      if ((rc = update_llr(c, priors, stream)) || (rc = update_masks(c, p, stream))) break;
      Plan pl;
      if ((rc = make_plan(c, p, shots, &pl))) break;
      max_w = pl.grid[MODE_MAIN] / c->cus;
    }
    for (int w = max_w; w >= 1 && !rc; w = w > 2 ? w - 2 : w - 1) {
      {
        std::lock_guard<std::mutex> lk(c->mu);
        c->tuned_D = ds[i];
        c->tuned_wpc = w;
      }
      // one untimed call, then the best of `reps`
      float t_best = 0.f;
      for (int r = 0; r <= reps && !rc; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(BPSF_EDEVICE, "event record"); break; }
        rc = bpsf_decode(c, syndromes, priors, shots, p, static_cast<uint8_t*>(corr.p), static_cast<uint8_t*>(conv.p),
                         static_cast<int32_t*>(it.p), stream);
        if (rc) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(BPSF_EDEVICE, "event wait");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 && (t_best == 0.f || ms < t_best)) t_best = ms;
      }
      if (rc) break;
      ++tried;
      if (best == 0.f || t_best < best) { best = t_best; best_D = ds[i]; best_w = w; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(c->mu);
  if (rc) {
    c->tuned_D = saved_D;
    c->tuned_wpc = saved_w;
    return rc;
  }
  c->tuned_D = best_D;
  c->tuned_wpc = best_w;
  out->decodes_per_wave = best_D;
  out->waves_per_cu = best_w;
  out->ms = best;
  out->candidates = tried;
  return 0;
}

int bpsf_reserve(bpsf_code c, int64_t shots, const bpsf_params* p)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (shots < 1 || shots > 0x7fffffffLL) return fail(BPSF_EINVAL, "shots must be in 1..2^31-1");
  std::lock_guard<std::mutex> lk(c->mu);
  Plan pl;
  // the tile of a call of `shots`, and those of the largest calls that take
  // the small family (more record words per shot)
  if ((rc = make_plan(c, p, shots, &pl))) return rc;
  for (int D = 1; D <= MAX_D && !rc; D *= 2) rc = make_plan(c, p, std::min(shots, SMALL_CALL_SHOTS_PER_D * D), &pl);
  return rc;
}

int bpsf_mix_reserve(bpsf_mix m, int64_t shots, const bpsf_params* p)
{
  if (!m) return fail(BPSF_EINVAL, "mix is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (shots < 1 || shots > 0x7fffffffLL) return fail(BPSF_EINVAL, "shots must be in 1..2^31-1");
  if (p->k > 16) return fail(BPSF_ENOTSUP, "mixed-code calls take |Phi| up to 16");
  std::lock_guard<std::mutex> lk(m->mu);
  int stride = 0;
  if ((rc = mix_stride_max(m, shots, p, &stride))) return rc;
  const size_t n = (size_t)shots;
  if (m->lists.ensure(sizeof(int32_t) * n * m->n) || m->rec_lists.ensure(sizeof(int32_t) * n * m->n) ||
      m->records.ensure(sizeof(int32_t) * n * (size_t)stride) || m->keys.ensure(sizeof(unsigned long long) * n) ||
      m->counters.ensure(sizeof(unsigned long long) * ((size_t)CNT_WORDS * m->n + MIX_WORDS)))
    return fail(BPSF_ENOMEM, "scratch for %lld shots", (long long)shots);
  // the corrections a call of the small form keeps: every code's region at
  // the most lanes a decode can have
  if (p->k > 0) {
    int64_t trials = 1;
    for (int i = 0; i < m->n; ++i) {
      TileDesc t;
      Args a;
      if (pick_tile(m->codes[i], &t)) return fail(BPSF_ENOTSUP, "code %d has no kernel tile", i);
      if ((rc = fill_code_args(m->codes[i], p, t, &a))) return rc;
      trials = std::max<int64_t>(trials, a.n_trials);
    }
    const size_t per_rec = sizeof(uint32_t) * (size_t)trials * 64 * (size_t)m->n;
    const int64_t recs = std::min<int64_t>(std::min(shots, SMALL_CALL_SHOTS), (int64_t)(TRIAL_BITS_MAX / per_rec));
    if (recs > 0 && m->trial_bits.ensure(per_rec * (size_t)recs, TRIAL_BITS_MAX))
      return fail(BPSF_ENOMEM, "trial corrections of %lld records", (long long)recs);
  }
  return 0;
}

}  // extern "C"

namespace {

int set_table(bpsf_code c, const void* masks, int64_t n_trials, int64_t stride, bool wide)
{
  if (!c) return fail(BPSF_EINVAL, "code is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  if (!masks) {
    c->table = nullptr;
    c->table_n = c->table_stride = 0;
    c->table64 = false;
    return 0;
  }
  if (n_trials < 1 || n_trials > 0x7fffffffLL) return fail(BPSF_EINVAL, "n_trials must be in 1..2^31-1");
  if (stride != 0 && stride != n_trials) return fail(BPSF_EINVAL, "stride must be 0 or n_trials");
  c->table = static_cast<const uint32_t*>(masks);
  c->table_n = n_trials;
  c->table_stride = stride;
  c->table64 = wide;
  return 0;
}

}  // namespace

extern "C" {

int bpsf_set_trial_table(bpsf_code c, const uint32_t* masks, int64_t n_trials, int64_t stride)
{
  return set_table(c, masks, n_trials, stride, false);
}

int bpsf_set_trial_table64(bpsf_code c, const uint64_t* masks, int64_t n_trials, int64_t stride)
{
  return set_table(c, masks, n_trials, stride, true);
}

}  // extern "C"

// Library-internal entry points of the request loop (bpsf_internal.h).
int bpsf::decode_in(bpsf_code c, const uint8_t* syndromes, const double* priors, int64_t shots,
                    const bpsf_params* p, uint8_t* corrections, uint8_t* converged, int32_t* iterations,
                    void* stream, void* scratch, size_t scratch_bytes)
{
  if (!scratch) return fail(BPSF_EINVAL, "NULL scratch");
  FixedScratch fx;
  fx.base = scratch;
  fx.bytes = scratch_bytes;
  fx.keep = true;   // the request loop leaves room for kept trial corrections
  return decode_call(c, syndromes, priors, shots, p, corrections, converged, iterations, stream, &fx);
}

int bpsf::mix_scratch_stride(bpsf_mix m, const bpsf_params* p, int* out)
{
  if (!m || !p || !out) return fail(BPSF_EINVAL, "NULL argument");
  int rc = check_params(p);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  // the same for every call size: the probes of mix_stride_max cover the
  // mixed tile and both single-code tiles whatever the size
  return mix_stride_max(m, SMALL_CALL_SHOTS, p, out);
}

size_t bpsf::mix_scratch_size(int n_codes, int64_t shots, int stride)
{
  return mix_fixed_bytes(n_codes, std::max<int64_t>(shots, 1), stride);
}

int bpsf::mix_scratch_bytes(bpsf_mix m, int64_t shots, const bpsf_params* p, size_t* out)
{
  if (!m || !p || !out) return fail(BPSF_EINVAL, "NULL argument");
  int rc = check_params(p);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(m->mu);
  int stride = 0;
  if ((rc = mix_stride_max(m, std::max<int64_t>(shots, 1), p, &stride))) return rc;
  *out = mix_fixed_bytes(m->n, std::max<int64_t>(shots, 1), stride);
  return 0;
}

int bpsf::mix_decode_grouped_in(bpsf_mix m, const int64_t* counts, const uint8_t* syndromes, int64_t syn_stride,
                                const double* const* priors, const bpsf_params* p, uint8_t* corrections,
                                int64_t corr_stride, uint8_t* converged, int32_t* iterations, void* stream,
                                void* scratch, size_t scratch_bytes)
{
  if (!m || !counts || !scratch) return fail(BPSF_EINVAL, "NULL argument");
  int64_t shots = 0;
  for (int i = 0; i < m->n; ++i) {
    if (counts[i] < 0) return fail(BPSF_EINVAL, "counts[%d] < 0", i);
    shots += counts[i];
  }
  FixedScratch fx;
  fx.base = scratch;
  fx.bytes = scratch_bytes;
  fx.keep = true;   // the request loop leaves room for kept trial corrections
  return mix_decode(m, nullptr, counts, syndromes, syn_stride, priors, shots, p, corrections, corr_stride, converged,
                    iterations, stream, &fx);
}
