// Where the sparse family keeps a code's messages in LDS, and in which order
// each check reads its row (host code only).
//
// None of these choices changes a result: the cells of a column stay in the
// caller's check order, which is the order of the bit phase's sums, and a
// check's minima and sign parity do not depend on the order of its row.
//
//   1. Checks and bits are renumbered by weight (ties by index), so that the
//      64 rows or columns a wave handles together have nearly equal weights.
//   2. Columns take consecutive cells in that order, each padded to an odd
//      length when room allows: the 32 lanes of a half-wave reading position
//      j of their columns then hit 32 distinct banks (bit phase). Within a
//      class of equal weight, which column sits in which slot is free; a local
//      search over swaps evens out, for every half-wave group of 32 checks,
//      how many of the group's cells fall in each bank.
//   3. The order of a row is a proper edge colouring of the bipartite
//      multigraph (checks of the group) x (banks), one edge per cell, colour =
//      position. With at least as many positions as the largest row weight
//      and the largest bank load of the group (Koenig's edge-colouring
//      theorem), the group's reads at every position hit distinct banks. A
//      row shorter than the position count reads +inf pad cells of lanes of
//      its own half-wave, taken in the banks left free at that position.
//
// LDS model (measured on gfx950 with 32-bit accesses at chosen lane
// patterns): 32 banks of 4 bytes; a half-wave's read takes as many cycles as
// the largest number of distinct addresses in one bank, a write at least two.
#include "bpsf_sparse_layout.h"

#include <algorithm>
#include <numeric>

namespace bpsf {

namespace {

constexpr int BANKS = 32;

// Marsaglia's xorshift64 (shifts 13, 7, 17) from a fixed seed: the layout is
// a function of the code alone.
struct Xorshift64 {
  uint64_t s = 0x9e3779b97f4a7c15ull;
  uint64_t next()
  {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
  }
  uint32_t below(uint32_t n) { return (uint32_t)(((next() >> 32) * (uint64_t)n) >> 32); }
};

// Places the columns of every weight class in the class's slots so that the
// summed excess of the (group, bank) cell counts over the groups' position
// counts is small: proposals swap two columns of one class and are kept when
// the excess does not grow. Stops at zero excess or after 64 proposals per
// column. Returns the excess left.
int balance_columns(const std::vector<std::vector<int>>& col_rows, const std::vector<int>& grp,
                    const std::vector<int>& cap, const std::vector<uint32_t>& colptr, std::vector<int>& col_of)
{
  const int N = (int)col_of.size();
  const int G = (int)cap.size();
  std::vector<int> load((size_t)G * BANKS, 0);
  for (int s = 0; s < N; ++s) {
    const std::vector<int>& rows = col_rows[(size_t)col_of[(size_t)s]];
    for (size_t k = 0; k < rows.size(); ++k)
      ++load[(size_t)grp[(size_t)rows[k]] * BANKS + (colptr[(size_t)s] + k) % BANKS];
  }
  auto excess = [&](int i, int v) { return std::max(0, v - cap[(size_t)(i / BANKS)]); };
  int total = 0;
  for (int i = 0; i < G * BANKS; ++i) total += excess(i, load[(size_t)i]);
  // the slots of a weight class are consecutive
  std::vector<int> lo((size_t)N), hi((size_t)N);
  for (int s = 0; s < N;) {
    int e = s;
    while (e < N && col_rows[(size_t)col_of[(size_t)e]].size() == col_rows[(size_t)col_of[(size_t)s]].size()) ++e;
    for (int q = s; q < e; ++q) {
      lo[(size_t)q] = s;
      hi[(size_t)q] = e;
    }
    s = e;
  }
  Xorshift64 rng;
  std::vector<int> idx, dv;   // (group, bank) entries a proposal changes, and by how much
  auto touch = [&](int i, int d) {
    for (size_t q = 0; q < idx.size(); ++q)
      if (idx[q] == i) {
        dv[q] += d;
        return;
      }
    idx.push_back(i);
    dv.push_back(d);
  };
  const long long proposals = 64LL * N;
  for (long long it = 0; it < proposals && total > 0; ++it) {
    const int a = (int)rng.below((uint32_t)N);
    const int n = hi[(size_t)a] - lo[(size_t)a];
    if (n < 2) continue;
    const int b = lo[(size_t)a] + (int)rng.below((uint32_t)n);
    if (b == a) continue;
    const std::vector<int>& ra = col_rows[(size_t)col_of[(size_t)a]];
    const std::vector<int>& rb = col_rows[(size_t)col_of[(size_t)b]];
    idx.clear();
    dv.clear();
    for (size_t k = 0; k < ra.size(); ++k) {
      const int ba = (int)((colptr[(size_t)a] + k) % BANKS), bb = (int)((colptr[(size_t)b] + k) % BANKS);
      const int ga = grp[(size_t)ra[k]] * BANKS, gb = grp[(size_t)rb[k]] * BANKS;
      touch(ga + ba, -1);
      touch(ga + bb, +1);
      touch(gb + bb, -1);
      touch(gb + ba, +1);
    }
    int delta = 0;
    for (size_t q = 0; q < idx.size(); ++q)
      delta += excess(idx[q], load[(size_t)idx[q]] + dv[q]) - excess(idx[q], load[(size_t)idx[q]]);
    if (delta > 0) continue;
    for (size_t q = 0; q < idx.size(); ++q) load[(size_t)idx[q]] += dv[q];
    std::swap(col_of[(size_t)a], col_of[(size_t)b]);
    total += delta;
  }
  return total;
}

// A proper edge colouring with D colours of the bipartite multigraph whose
// edge e joins row erow[e] (< n) and bank ebank[e] (< 32); D must be at least
// every row's and every bank's degree. Each edge in turn takes the first
// colour a free at its row; when a is taken at its bank, the path from the
// bank that alternates a and b (the bank's first free colour) has its two
// colours swapped first. That path cannot reach the row (a is free there), so
// afterwards a is free at both ends. Returns false if D is too small.
bool colour_edges(const std::vector<int>& erow, const std::vector<int>& ebank, int n, int D, std::vector<int>& col)
{
  const size_t E = erow.size();
  col.assign(E, -1);
  std::vector<int> at_row((size_t)n * D, -1), at_bank((size_t)BANKS * D, -1), path;
  for (size_t e = 0; e < E; ++e) {
    const int u = erow[e], v = ebank[e];
    int a = 0, b = 0;
    while (a < D && at_row[(size_t)u * D + a] >= 0) ++a;
    while (b < D && at_bank[(size_t)v * D + b] >= 0) ++b;
    if (a == D || b == D) return false;
    if (at_bank[(size_t)v * D + a] >= 0) {
      path.clear();
      int x = v, c = a;
      bool at_bank_side = true;
      for (;;) {
        const int m = at_bank_side ? at_bank[(size_t)x * D + c] : at_row[(size_t)x * D + c];
        if (m < 0) break;
        path.push_back(m);
        x = at_bank_side ? erow[(size_t)m] : ebank[(size_t)m];
        at_bank_side = !at_bank_side;
        c = c == a ? b : a;
      }
      for (int m : path) {
        at_row[(size_t)erow[(size_t)m] * D + col[(size_t)m]] = -1;
        at_bank[(size_t)ebank[(size_t)m] * D + col[(size_t)m]] = -1;
      }
      for (int m : path) {
        col[(size_t)m] = col[(size_t)m] == a ? b : a;
        at_row[(size_t)erow[(size_t)m] * D + col[(size_t)m]] = m;
        at_bank[(size_t)ebank[(size_t)m] * D + col[(size_t)m]] = m;
      }
    }
    col[e] = a;
    at_row[(size_t)u * D + a] = (int)e;
    at_bank[(size_t)v * D + a] = (int)e;
  }
  return true;
}

}  // namespace

void sparse_tables(const int32_t* row_ptr, const int32_t* col_idx, int M, int N, const SparseDesc& d,
                   SparseTables* out)
{
  SparseTables& t = *out;
  const int T = 64 * d.NW;
  std::vector<int> colw((size_t)N, 0);
  for (int e = 0; e < row_ptr[M]; ++e) ++colw[(size_t)col_idx[e]];
  auto roww = [&](int r) { return row_ptr[r + 1] - row_ptr[r]; };

  // 1. renumbering by weight
  std::vector<int> rperm((size_t)M), cperm((size_t)N), rinv((size_t)M), cinv((size_t)N);
  std::iota(rperm.begin(), rperm.end(), 0);
  std::iota(cperm.begin(), cperm.end(), 0);
  std::stable_sort(rperm.begin(), rperm.end(), [&](int x, int y) { return roww(x) < roww(y); });
  std::stable_sort(cperm.begin(), cperm.end(), [&](int x, int y) { return colw[(size_t)x] < colw[(size_t)y]; });
  for (int i = 0; i < M; ++i) rinv[(size_t)rperm[(size_t)i]] = i;

  // 2. column cells: one more for a column of even weight, when room allows
  auto col_cells = [&](int w, bool pad) { return (uint32_t)(pad && (w % 2 == 0) ? w + 1 : w); };
  uint32_t padded = 0;
  for (int v = 0; v < N; ++v) padded += col_cells(colw[(size_t)v], true);
  const bool pad_cols = (int64_t)padded + d.DVMAX + (int64_t)T * d.CPT <= 65535;
  std::vector<uint32_t> colptr((size_t)N + 1, 0);
  for (int v = 0; v < N; ++v) colptr[(size_t)v + 1] = colptr[(size_t)v] + col_cells(colw[(size_t)cperm[(size_t)v]], pad_cols);
  t.cells = (int)colptr[(size_t)N];

  // the caller's checks of every caller's bit, ascending (a column's cells)
  std::vector<std::vector<int>> col_rows((size_t)N);
  for (int r = 0; r < M; ++r)
    for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) col_rows[(size_t)col_idx[e]].push_back(r);
  // half-wave groups of 32 internal checks; a group reads as many positions
  // as the largest weight in its wave (64 checks), at least
  const int G = (M + 31) / 32;
  std::vector<int> grp((size_t)M), cap((size_t)G, 0);
  for (int r = 0; r < M; ++r) grp[(size_t)r] = rinv[(size_t)r] / 32;
  for (int ri = 0; ri < M; ++ri) {
    const int w0 = (ri / 64) * 2;
    for (int g = w0; g < std::min(G, w0 + 2); ++g) cap[(size_t)g] = std::max(cap[(size_t)g], roww(rperm[(size_t)ri]));
  }
  t.overflow = balance_columns(col_rows, grp, cap, colptr, cperm);
  for (int i = 0; i < N; ++i) cinv[(size_t)cperm[(size_t)i]] = i;

  // cells of every internal check; the internal check of every cell
  std::vector<std::vector<uint32_t>> rcells((size_t)M);
  t.echk.assign((size_t)(t.cells > 0 ? t.cells : 1), 0);
  for (int s = 0; s < N; ++s) {
    const std::vector<int>& rows = col_rows[(size_t)cperm[(size_t)s]];
    for (size_t k = 0; k < rows.size(); ++k) {
      const uint32_t cell = colptr[(size_t)s] + (uint32_t)k;
      const int ri = rinv[(size_t)rows[k]];
      rcells[(size_t)ri].push_back(cell);
      t.echk[cell] = (uint16_t)ri;
    }
  }

  // 3. row orders, group by group
  auto pad_cell = [&](int ri) { return (uint32_t)(t.cells + d.DVMAX + (ri % T) * d.CPT + ri / T); };
  t.roff.assign((size_t)M * d.WMAX, 0);
  t.rw.assign((size_t)M, 0);
  t.extra_positions = 0;
  t.folded = 0;
  std::vector<int> erow, ebank, col, pos;
  std::vector<uint32_t> ecell;
  for (int g = 0; g < G; ++g) {
    const int r0 = 32 * g, n = std::min(32, M - r0);
    erow.clear();
    ebank.clear();
    ecell.clear();
    int D = cap[(size_t)g];
    int load[BANKS] = {0};
    for (int l = 0; l < n; ++l) {
      D = std::max(D, (int)rcells[(size_t)(r0 + l)].size());
      for (uint32_t cell : rcells[(size_t)(r0 + l)]) {
        erow.push_back(l);
        ebank.push_back((int)(cell % BANKS));
        ecell.push_back(cell);
        ++load[cell % BANKS];
      }
    }
    for (int b = 0; b < BANKS; ++b) D = std::max(D, load[b]);
    t.extra_positions += D - cap[(size_t)g];
    // D bounds every degree, so the colouring cannot fail
    (void)colour_edges(erow, ebank, n, D, col);
    // at most WMAX positions: a colour past them moves to the row's first
    // free position (sharing a bank there)
    const int P = std::min(D, d.WMAX);
    pos.assign((size_t)n * P, -1);
    for (size_t e = 0; e < ecell.size(); ++e)
      if (col[e] >= 0 && col[e] < P) pos[(size_t)erow[e] * P + col[e]] = (int)ecell[e];
    for (size_t e = 0; e < ecell.size(); ++e) {
      if (col[e] >= 0 && col[e] < P) continue;
      int j = 0;
      while (pos[(size_t)erow[e] * P + j] >= 0) ++j;   // a row has at most WMAX cells
      pos[(size_t)erow[e] * P + j] = (int)ecell[e];
      ++t.folded;
    }
    // lanes of the half-wave past the last check read their own pad cells
    uint32_t idle = 0;
    for (int l = n; l < 32; ++l) idle |= 1u << (pad_cell(r0 + l) % BANKS);
    for (int j = 0; j < P; ++j) {
      uint32_t used = idle;
      for (int l = 0; l < n; ++l)
        if (pos[(size_t)l * P + j] >= 0) used |= 1u << ((uint32_t)pos[(size_t)l * P + j] % BANKS);
      for (int l = 0; l < n; ++l) {
        if (pos[(size_t)l * P + j] >= 0) continue;
        uint32_t cell = pad_cell(r0 + l);   // own pad unless a pad of the half-wave is in a free bank
        for (int q = 0; q < n; ++q) {
          const uint32_t pc = pad_cell(r0 + q);
          if (!((used >> (pc % BANKS)) & 1u)) {
            cell = pc;
            break;
          }
        }
        used |= 1u << (cell % BANKS);
        pos[(size_t)l * P + j] = (int)cell;
      }
    }
    for (int l = 0; l < n; ++l) {
      const int ri = r0 + l;
      for (int j = 0; j < d.WMAX; ++j)
        t.roff[(size_t)ri * d.WMAX + j] = (uint16_t)(j < P ? (uint32_t)pos[(size_t)l * P + j] : pad_cell(ri));
      t.rw[(size_t)ri] = (uint8_t)P;
    }
  }

  t.bits.resize((size_t)N);
  t.cperm.resize((size_t)N);
  t.cinv.resize((size_t)N);
  t.rperm.resize((size_t)M);
  for (int v = 0; v < N; ++v) {
    t.bits[(size_t)v] = colptr[(size_t)v] | ((uint32_t)colw[(size_t)cperm[(size_t)v]] << 16);
    t.cperm[(size_t)v] = (uint16_t)cperm[(size_t)v];
    t.cinv[(size_t)v] = (uint16_t)cinv[(size_t)v];
  }
  for (int i = 0; i < M; ++i) t.rperm[(size_t)i] = (uint16_t)rperm[(size_t)i];
}

}  // namespace bpsf
