// Kernel families of the BP-SF decoder and the LDS layout they imply.
// Shared by the device code and the host runtime (library-internal).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace bpsf {

// A family fixes, at compile time, the items every lane owns (IC checks and
// IV bits), the ELL row width W and the column weight DV. The number of
// decodes a wave runs at once (D, a power of two from 1 to 16, so G = 64 / D
// lanes per decode) is a launch parameter: a code with M checks and N bits
// fits when M <= G * IC and N <= G * IV.
//
// Messages of slot d sit at stride MS = G * IC inside each edge position of
// CI = 64 * IC entries, so CI does not depend on D. A lane's check items sit
// at IC * lane + k: with IC odd the 32 lanes of a half-wave hit 32 distinct
// banks in the check phase. With IC = 1 (mod 8) also MS = G (mod 32) for
// every G >= 4, which keeps the bit-phase gathers of the slots sharing a
// half-wave apart; the small family (IC = 3) runs at G >= 16.
// ints per ring entry header: shot (two words for the first BP), record,
// trial, first-BP iterations
constexpr int RING_META = 5;

template <int IC_, int IV_, int W_, int DV_>
struct Family {
  static constexpr int IC = IC_, IV = IV_, W = W_, DV = DV_;
  static constexpr int CI = 64 * IC;   // message entries per edge position
  static constexpr int PL = 8;         // bit planes of flip_count
  static constexpr int META = RING_META;
  static constexpr int KMAX = 16;      // largest |Phi|
  static_assert(IC % 2 == 1, "IC odd keeps check-phase accesses free of bank conflicts");
  static_assert(IC <= 16 && IV <= 32, "items per lane must fit the 16-bit column masks and 32-bit bit masks");
  static_assert(W >= 2 && DV >= 1, "row weight >= 2");
};

// Compiled families (IC, IV, W, DV): row weight 6 / column weight 3 (the
// bivariate-bicycle and coprime-BB codes), row weight 10 / column weight 5
// (the generalized-bicycle code of Appendix A), and a small row-weight-6
// family with a third of the items per lane, for calls too small to fill the
// GPU, where the time of one iteration of one wave is the latency.
#define BPSF_FAMILY_LIST(X) \
  X(9, 18, 6, 3)            \
  X(9, 9, 10, 5)            \
  X(3, 5, 6, 3)

constexpr int MAX_D = 16;

struct TileDesc {
  int fam;   // index into BPSF_FAMILY_LIST
  int D;     // decodes per wave
};

struct FamilyDesc {
  int IC, IV, W, DV;
};

struct LdsLayout {
  uint32_t msg, resid, chk, lrow, ring_meta, ring_tb, ring_syn, lpost, ellw, total;
};

__host__ __device__ inline uint32_t lds_align16(uint32_t o) { return (o + 15u) & ~15u; }

// Byte offsets of the LDS regions of one wave: a family with CI entries per
// edge position, a code with M checks and N bits, D decodes per wave; `lrow`
// (the channel LLR of every edge, used to reset messages) only when the
// priors are not uniform.
__host__ __device__ inline LdsLayout lds_layout(int real_bytes, int W, int CI, int M, int N, int DV, int D,
                                                bool uniform, int META, bool layered = false, int IV = 0)
{
  LdsLayout L;
  const int ring = 2 * D;
  uint32_t o = 0;
  L.msg = o;                                           // W x CI messages + 64-entry sink
  o += (uint32_t)real_bytes * (uint32_t)(W * CI + 64);
  o = lds_align16(o);
  L.resid = o;                                         // u = H e, 16 bits per lane: bit k = check item k
  o += 2u * 64u;
  o = lds_align16(o);
  L.chk = o;                                           // checks of every bit (u16)
  o += 2u * (uint32_t)(N * DV);
  o = lds_align16(o);
  L.lrow = o;                                          // [W][M] channel LLR of the bit on each edge
  if (!uniform) o += (uint32_t)real_bytes * (uint32_t)(W * M);
  o = lds_align16(o);
  L.ring_meta = o;                                     // task headers
  o += 4u * (uint32_t)(ring * META);
  L.ring_tb = o;                                       // trial bits of every lane of an entry
  o += 4u * (uint32_t)(ring * (64 / D));
  L.ring_syn = o;                                      // syndrome bits of every lane of an entry (u16)
  o += 2u * (uint32_t)(ring * (64 / D));
  o = lds_align16(o);
  // layered schedule: the posterior of every bit of every slot, and the bit
  // of every (check, position)
  L.lpost = o;
  if (layered) o += (uint32_t)real_bytes * 64u * (uint32_t)IV;
  o = lds_align16(o);
  L.ellw = o;
  if (layered) o += 2u * (uint32_t)(M * W);
  L.total = lds_align16(o);
  return L;
}

// Wide families: one decode per workgroup of NW waves (G = 64 NW lanes),
// lane g owning checks g*IC + k and bits g + G*k; rows and columns may be
// irregular, padded to W and DV. For codes too large for one wave.
template <int NW_, int IC_, int IV_, int W_, int DV_>
struct WideFamily {
  static constexpr int NW = NW_, IC = IC_, IV = IV_, W = W_, DV = DV_;
  static constexpr int G = 64 * NW;    // lanes of a decode
  static constexpr int MP = G * IC;    // padded checks (message stride per edge position)
  static constexpr int PL = 8, KMAX = 16;
  static_assert(IC % 2 == 1, "an odd IC keeps check-phase accesses free of bank conflicts");
  static_assert(IC <= 16 && IV <= 32 && IV * DV <= 64, "items must fit the 16/32/64-bit masks");
};

// Compiled wide families (NW, IC, IV, W, DV): up to 960 checks and 2688 bits
// of row weight <= 8 and column weight <= 3 (the phenomenological
// [[144,12,12]] matrix over 12 rounds is 864 x 2592).
#define BPSF_WIDE_LIST(X) \
  X(3, 5, 14, 8, 3)

struct WideDesc {
  int NW, IC, IV, W, DV;
};

struct WideLayout {
  uint32_t msg, zero, dummy, resid, red, task, flags, total;
};

// LDS of a wide-family workgroup.
__host__ __device__ inline WideLayout wide_layout(int real_bytes, int W, int MP, int NW)
{
  WideLayout L;
  uint32_t o = 0;
  L.msg = o;                                           // W x MP messages
  o += (uint32_t)real_bytes * (uint32_t)(W * MP);
  o = lds_align16(o);
  L.zero = o;                                          // reads of missing edges: 0
  o += 16u;
  L.dummy = o;                                         // writes of missing edges, one cell per lane
  o += 4u * 64u * (uint32_t)NW * (real_bytes == 8 ? 2u : 1u);
  o = lds_align16(o);
  L.resid = o;                                         // u = H e, one word per padded check
  o += 4u * (uint32_t)MP;
  o = lds_align16(o);
  L.red = o;                                           // per-wave partial reductions
  o += 4u * (uint32_t)NW;
  o = lds_align16(o);
  L.task = o;                                          // claimed task, record, trial, skip
  o += 8u * 4u;
  L.flags = o;                                         // per-wave unsatisfied flags + stop, two iterations
  o += 4u * 2u * (uint32_t)(NW + 1);
  L.total = lds_align16(o);
  return L;
}

struct Args;
struct MixArgs;
struct BucketArgs;
int family_count();
FamilyDesc family_desc(int fam);
// what = 0: launch; what = 1: *out = resident blocks per CU
int tile_dispatch(int what, const TileDesc& t, bool fp64, bool uniform_llr, int mode, bool trace,
                  const Args& a, size_t lds_bytes, int grid, void* stream, int* out, bool layered = false);
// every code of m belongs to family fam; small: the form for calls of at most
// 65536 shots (first chunks by rank, kept trial corrections)
int mixed_dispatch(int what, int fam, bool fp64, bool uniform_llr, bool small, int mode, const MixArgs& m,
                   size_t lds_bytes, int grid, void* stream, int* out);
int bucket_launch(const BucketArgs& b, void* stream);
int wide_count();
WideDesc wide_desc(int fam);
int wide_dispatch(int what, int fam, bool fp64, int mode, const Args& a, size_t lds_bytes, int grid, void* stream,
                  int* out);
int reset_counters(unsigned long long* c, int n, void* stream);   // zero n words

}  // namespace bpsf
