// Sparse kernel family (large irregular matrices): compile-time shapes, LDS
// layout and dispatch. Separate from bpsf_tiles.h so that the one-wave and
// wide families do not depend on it.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "bpsf_tiles.h"

namespace bpsf {

// Large irregular matrices (circuit-level detector error models): one decode
// per workgroup of NW waves, T = 64 NW threads; thread g owns the checks
// g + T i (i < CPT) and the bits g + T i (i < BPT); rows of weight <= WMAX,
// columns of weight <= DVMAX; messages stored once per edge, in column-major
// order, float only.
template <int NW_, int CPT_, int WMAX_, int BPT_, int DVMAX_>
struct SparseFamily {
  static constexpr int NW = NW_, CPT = CPT_, WMAX = WMAX_, BPT = BPT_, DVMAX = DVMAX_;
  static constexpr int T = 64 * NW;
  static constexpr int PL = 8, KMAX = 64;   // |Phi| up to 64 (records hold Phi only)
  static_assert(BPT <= 32 && WMAX % 2 == 0, "bit masks are 32 bits; row offsets come in pairs");
};

// Compiled sparse families (NW, CPT, WMAX, BPT, DVMAX): up to 1024 checks and
// 9216 bits (the [[144,12,12]] memory circuit over 12 rounds gives 936
// detectors and about 8,800 mechanisms, rows of weight <= 41, columns <= 9).
// Sixteen waves of one check and nine bits per thread: they hide LDS latency
// better than eight waves of two checks and eighteen bits, which cover the
// same shapes (measured: the first-BP phase of that model ran 1.35x faster).
#define BPSF_SPARSE_LIST(X) \
  X(16, 1, 48, 9, 10)

struct SparseDesc {
  int NW, CPT, WMAX, BPT, DVMAX;
};

struct SparseLayout {
  uint32_t msg, ubits, sbits, red, task, flags, total;
};

// LDS of a sparse-family workgroup for E edges and M checks: the cells (E
// messages, then DVMAX cells read past the last column, then one pad cell per
// check slot of every thread, T CPT of them), u = H e and s as bit vectors,
// reductions.
__host__ __device__ inline SparseLayout sparse_layout(int E, int M, int NW, int DVMAX, int CPT)
{
  SparseLayout L;
  uint32_t o = 0;
  L.msg = o;
  o += 4u * (uint32_t)(E + DVMAX + 64 * NW * CPT);
  o = lds_align16(o);
  L.ubits = o;
  o += 4u * (uint32_t)((M + 31) / 32);
  o = lds_align16(o);
  L.sbits = o;
  o += 4u * (uint32_t)((M + 31) / 32);
  o = lds_align16(o);
  L.red = o;
  o += 4u * (uint32_t)NW;
  o = lds_align16(o);
  L.task = o;
  o += 8u * 4u;
  L.flags = o;
  o += 4u * 2u * (uint32_t)(NW + 1);
  L.total = lds_align16(o);
  return L;
}

// Set by the host in Args::flags (above the caller's flags) when trial_masks
// holds 64-bit masks.
constexpr int SPARSE_FLAG_MASKS64 = 1 << 16;

struct Args;
int sparse_count();
SparseDesc sparse_desc(int fam);
int sparse_dispatch(int what, int fam, int mode, const Args& a, size_t lds_bytes, int grid, void* stream, int* out);

}  // namespace bpsf
