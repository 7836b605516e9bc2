// Tile shapes of the BP-SF kernel and the LDS layout they imply.
// Shared by the device code and the host runtime (library-internal).
#pragma once

#include <stdint.h>

namespace bpsf {

// Slot stride: at least G*IC entries and congruent to G modulo 32, so the 32
// lanes of each half-wave hit 32 distinct banks in the check phase.
constexpr int slot_stride_c(int G, int IC)
{
  int ms = G * IC;
  const int want = G % 32;
  while (ms % 32 != want) ++ms;
  return ms;
}

// D: decodes (slots) per wave; IC / IV: check / bit items per lane;
// W: ELL row width; DV: column weight.
template <int D_, int IC_, int IV_, int W_, int DV_>
struct TileShape {
  static constexpr int D = D_, IC = IC_, IV = IV_, W = W_, DV = DV_;
  static constexpr int G = 64 / D;                  // lanes per slot
  static constexpr int LG = G == 64 ? 6 : G == 32 ? 5 : G == 16 ? 4 : G == 8 ? 3 : G == 4 ? 2 : G == 2 ? 1 : 0;
  static constexpr int RING = 2 * D;                // prefetched tasks
  static constexpr int PL = 8;                      // bit planes of flip_count
  static constexpr int META = 8;                    // ints per ring entry header
  static constexpr int KMAX = 16;                   // largest |Phi|
  static constexpr int KG = (KMAX + G - 1) / G;     // Phi entries per lane
  static constexpr int MS = slot_stride_c(G, IC);   // message entries per slot and edge position
  static constexpr int CI = D * MS;                 // entries per edge position
  static constexpr int MSB = (MS + 63) / 64;        // 64-lane blocks covering one slot's stride
  static_assert(D * G == 64, "D must divide 64");
  static_assert(IC <= 32 && IV <= 32, "items per lane must fit a 32-bit mask");
  static_assert(W >= 2 && DV >= 1, "row weight >= 2");
};

struct TileDesc {
  int D, IC, IV, W, DV;
};

// Compiled tiles (D, IC, IV, W, DV).
#define BPSF_TILE_LIST(X) \
  X(16, 9, 18, 6, 3)      \
  X(8, 9, 18, 6, 3)       \
  X(4, 9, 18, 6, 3)       \
  X(8, 6, 12, 6, 3)       \
  X(8, 7, 14, 6, 3)

struct LdsLayout {
  uint32_t msg, resid, chk, ring_meta, ring_tv, ring_syn, total;
};

__host__ __device__ inline uint32_t lds_align16(uint32_t o) { return (o + 15u) & ~15u; }

// Byte offsets of the LDS regions of one wave.
__host__ __device__ inline LdsLayout lds_layout(int real_bytes, int W, int CI, int RW, int N, int DV, int RING,
                                                int META, int KMAX, int G)
{
  LdsLayout L;
  uint32_t o = 0;
  L.msg = o;                                           // W x CI messages + 64-entry sink
  o += (uint32_t)real_bytes * (uint32_t)(W * CI + 64);
  o = lds_align16(o);
  L.resid = o;                                         // u = H e, one word per check of every slot
  o += 4u * (uint32_t)RW;
  o = lds_align16(o);
  L.chk = o;                                           // checks of every bit (u16)
  o += 2u * (uint32_t)(N * DV);
  o = lds_align16(o);
  L.ring_meta = o;
  o += 4u * (uint32_t)(RING * META);
  L.ring_tv = o;                                       // trial bits per lane of every entry
  o += 4u * (uint32_t)(RING * (KMAX > G ? KMAX : G));
  L.ring_syn = o;
  o += 4u * (uint32_t)(RING * G);
  L.total = lds_align16(o);
  return L;
}

struct Args;
int tile_dispatch(int what, const TileDesc& t, bool fp64, bool uniform_llr, int mode, bool trace,
                  const Args& a, int grid, void* stream, int* out);
int reset_counters(unsigned long long* c, void* stream);

}  // namespace bpsf
