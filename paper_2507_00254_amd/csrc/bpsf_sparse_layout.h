// Host side of the sparse kernel family: where a code's messages sit in LDS
// and in which order each check reads its row. Pure host code (no device
// calls), so it runs, and is tested, without a GPU.
#pragma once

#include <stdint.h>

#include <vector>

#include "bpsf_sparse.h"

namespace bpsf {

struct SparseTables {
  int cells = 0;                 // message cells: the columns, each padded to an odd length when room allows
  std::vector<uint16_t> roff;    // [M][WMAX] cell read at each position of an internal check's row
  std::vector<uint8_t> rw;       // [M] positions the check's half-wave reads (>= its weight)
  std::vector<uint16_t> echk;    // [cells] internal check of every cell (0 for padding)
  std::vector<uint32_t> bits;    // [N] internal bit: first cell | weight << 16
  std::vector<uint16_t> rperm;   // [M] caller's check of each internal check
  std::vector<uint16_t> cperm;   // [N] caller's bit of each internal bit
  std::vector<uint16_t> cinv;    // [N] internal bit of each caller's bit
  // how close the layout came to conflict-free row reads
  int overflow = 0;              // cells above their bank's share after the column placement
  int extra_positions = 0;       // positions added over all half-wave groups to fit every bank's load
  int folded = 0;                // cells moved to a position that shares its bank (only past WMAX positions)
};

// The tables of family d for the code given as CSR rows (ascending columns),
// already checked to fit the family. Deterministic: the same code gives the
// same tables.
void sparse_tables(const int32_t* row_ptr, const int32_t* col_idx, int M, int N, const SparseDesc& d,
                   SparseTables* out);

}  // namespace bpsf
