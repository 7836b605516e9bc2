// Sanitizer driver for the library's host runtime (test infrastructure):
// built from host-only compiles of the library's sources with
// AddressSanitizer and UndefinedBehaviorSanitizer, it drives every entry
// point of include/bpsf.h through its argument checks (the paths that run
// before any device work) and loads a code, which reaches the first device
// call (an error without a GPU). Any invalid access or undefined operation
// aborts the run.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/bpsf.h"

static int fails = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "line %d: expected %s (%s)\n", __LINE__, #cond, bpsf_last_error()); \
      ++fails;                                                         \
    }                                                                  \
  } while (0)

static bpsf_params params(int k = 6)
{
  bpsf_params p;
  memset(&p, 0, sizeof p);
  p.max_iter = 100;
  p.cand_max_iter = 20;
  p.k = k;
  p.w_max = 1;
  p.alpha = 0.625;
  return p;
}

int main()
{
  EXPECT(bpsf_last_error() != nullptr);
  // trial lists and parameter checks (no device)
  bpsf_params p = params();
  std::vector<uint32_t> masks(1 << 16);
  EXPECT(bpsf_num_trials(&p, masks.data(), (int64_t)masks.size()) == 64);
  p.cand_mode = BPSF_TRIALS_WEIGHT_LE;
  p.w_max = 3;
  p.k = 16;
  EXPECT(bpsf_num_trials(&p, masks.data(), 10) == 16 + 120 + 560);
  EXPECT(bpsf_num_trials(&p, nullptr, 0) == 696);
  const bpsf_params bad[] = {
      [] { bpsf_params q = params(); q.max_iter = 0; return q; }(),
      [] { bpsf_params q = params(); q.max_iter = 256; return q; }(),
      [] { bpsf_params q = params(); q.k = 17; return q; }(),
      [] { bpsf_params q = params(); q.k = -1; return q; }(),
      [] { bpsf_params q = params(); q.cand_max_iter = 4096; return q; }(),
      [] { bpsf_params q = params(); q.cand_mode = 7; return q; }(),
      [] { bpsf_params q = params(); q.cand_mode = BPSF_TRIALS_WEIGHT_LE; q.w_max = 7; return q; }(),
      [] { bpsf_params q = params(); q.select_mode = 3; return q; }(),
      [] { bpsf_params q = params(); q.alpha = -1.0; return q; }(),
      [] { bpsf_params q = params(); q.flags = 1 << 9; return q; }(),
      [] { bpsf_params q = params(); q.flags = BPSF_FLAG_PRUNE; return q; }(),
      [] { bpsf_params q = params(); q.precision = 5; return q; }(),
      [] { bpsf_params q = params(); q.cand_mode = BPSF_TRIALS_TABLE; return q; }(),
  };
  for (const bpsf_params& q : bad) EXPECT(bpsf_num_trials(&q, masks.data(), 4) == BPSF_EINVAL);
  EXPECT(bpsf_num_trials(nullptr, nullptr, 0) == BPSF_EINVAL);

  // malformed and unsupported matrices (checked before any device call)
  bpsf_code c = nullptr;
  const int32_t rp_ok[3] = {0, 2, 4}, ci_ok[4] = {0, 1, 1, 2};
  const int32_t rp_bad0[3] = {1, 2, 4}, rp_dec[3] = {0, 3, 2}, ci_range[4] = {0, 9, 1, 2}, ci_unsorted[4] = {1, 0, 1, 2};
  EXPECT(bpsf_load_code(rp_ok, ci_ok, 2, 3, nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_load_code(nullptr, ci_ok, 2, 3, &c) == BPSF_EINVAL && c == nullptr);
  EXPECT(bpsf_load_code(rp_bad0, ci_ok, 2, 3, &c) == BPSF_EINVAL);
  EXPECT(bpsf_load_code(rp_dec, ci_ok, 2, 3, &c) == BPSF_EINVAL);
  EXPECT(bpsf_load_code(rp_ok, ci_range, 2, 3, &c) == BPSF_EINVAL);
  EXPECT(bpsf_load_code(rp_ok, ci_unsorted, 2, 3, &c) == BPSF_EINVAL);
  EXPECT(bpsf_load_code(rp_ok, nullptr, 2, 3, &c) == BPSF_EINVAL);
  EXPECT(bpsf_load_code(rp_ok, ci_ok, 0, 3, &c) == BPSF_EINVAL);
  const int32_t rp_w1[3] = {0, 1, 3}, ci_w1[3] = {0, 1, 2};
  EXPECT(bpsf_load_code(rp_w1, ci_w1, 2, 3, &c) == BPSF_ENOTSUP);   // a check of weight 1
  std::vector<int32_t> rp_heavy(13), ci_heavy;   // a column of weight 12
  for (int r = 0; r < 12; ++r) {
    rp_heavy[r] = (int32_t)ci_heavy.size();
    ci_heavy.push_back(0);
    ci_heavy.push_back(1 + r);
  }
  rp_heavy[12] = (int32_t)ci_heavy.size();
  EXPECT(bpsf_load_code(rp_heavy.data(), ci_heavy.data(), 12, 13, &c) == BPSF_ENOTSUP);

  // a valid code: [[72,12,6]] H_X; without a GPU the load stops at its first device call
  {
    const int l = 6, m = 6, n = 36;
    std::vector<int32_t> rp(n + 1), ci;
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < m; ++j) {
        rp[i * m + j] = (int32_t)ci.size();
        std::vector<int32_t> row = {((i + 3) % l) * m + j, i * m + (j + 1) % m, i * m + (j + 2) % m,
                                    n + i * m + (j + 3) % m, n + ((i + 1) % l) * m + j, n + ((i + 2) % l) * m + j};
        for (size_t a = 0; a < row.size(); ++a)
          for (size_t b = a + 1; b < row.size(); ++b)
            if (row[b] < row[a]) std::swap(row[a], row[b]);
        ci.insert(ci.end(), row.begin(), row.end());
      }
    rp[n] = (int32_t)ci.size();
    const int rc = bpsf_load_code(rp.data(), ci.data(), n, 2 * n, &c);
    EXPECT(rc == BPSF_OK || rc == BPSF_EDEVICE);
    if (rc == BPSF_OK) bpsf_free_code(c);
    c = nullptr;
  }

  // an irregular matrix of the sparse family (columns of weight 2..6): its
  // LDS layout on the host, then a load (which computes the layout before its
  // first device call)
  {
    const int m = 900, n = 6000;
    std::vector<std::vector<int32_t>> rows(m);
    uint64_t x = 12345;
    auto next = [&]() { x = x * 6364136223846793005ull + 1442695040888963407ull; return (uint32_t)(x >> 33); };
    for (int v = 0; v < n; ++v) {
      const int w = 2 + (int)(next() % 5);
      std::vector<int> picked;
      while ((int)picked.size() < w) {
        const int r = (int)(next() % m);
        bool dup = false;
        for (int q : picked) dup = dup || q == r;
        if (!dup) picked.push_back(r);
      }
      for (int r : picked) rows[(size_t)r].push_back(v);
    }
    std::vector<int32_t> rp(1, 0), ci;
    int mm = 0;
    for (int r = 0; r < m; ++r) {
      if (rows[(size_t)r].size() < 2) continue;
      ci.insert(ci.end(), rows[(size_t)r].begin(), rows[(size_t)r].end());
      rp.push_back((int32_t)ci.size());
      ++mm;
    }
    int32_t info[BPSF_SPARSE_INFO_WORDS];
    EXPECT(bpsf_sparse_layout(rp.data(), ci.data(), mm, n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
           BPSF_EINVAL);
    EXPECT(bpsf_sparse_layout(rp.data(), ci.data(), mm, n, info, nullptr, nullptr, nullptr, nullptr, nullptr) == 0);
    EXPECT(info[0] >= 0);
    if (info[0] >= 0) {
      const int cells = info[1], wmax = info[2];
      std::vector<uint16_t> roff((size_t)mm * wmax), cperm(n), rperm(mm);
      std::vector<uint8_t> rw(mm);
      std::vector<uint32_t> bits(n);
      EXPECT(bpsf_sparse_layout(rp.data(), ci.data(), mm, n, info, roff.data(), rw.data(), bits.data(), cperm.data(),
                                rperm.data()) == 0);
      // every cell is read by exactly one check, once
      std::vector<int> reads((size_t)cells, 0);
      for (int r = 0; r < mm; ++r)
        for (int j = 0; j < rw[(size_t)r]; ++j)
          if (roff[(size_t)r * wmax + j] < cells) ++reads[roff[(size_t)r * wmax + j]];
      int edges = 0, bad = 0;
      for (int cell = 0; cell < cells; ++cell) {
        edges += reads[(size_t)cell];
        bad += reads[(size_t)cell] > 1;
      }
      EXPECT(edges == (int)ci.size() && bad == 0);
    }
    const int rc = bpsf_load_code(rp.data(), ci.data(), mm, n, &c);
    EXPECT(rc == BPSF_OK || rc == BPSF_EDEVICE);
    if (rc == BPSF_OK) bpsf_free_code(c);
    c = nullptr;
    // a code of another family has no sparse layout
    EXPECT(bpsf_sparse_layout(rp_ok, ci_ok, 2, 3, info, nullptr, nullptr, nullptr, nullptr, nullptr) == 0 &&
           info[0] == -1);
  }

  // every entry point with a NULL handle or argument
  bpsf_params q = params();
  bpsf_stats st;
  uint8_t u8[8] = {0};
  int32_t i32[8] = {0};
  int64_t i64[8] = {0};
  double d8[8] = {0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 0.01};
  float f4[4];
  EXPECT(bpsf_decode(nullptr, u8, d8, 1, &q, u8, u8, i32, nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_decode_noalloc(nullptr, u8, d8, 1, &q, u8, u8, i32, nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_reserve(nullptr, 10, &q) == BPSF_EINVAL);
  EXPECT(bpsf_last_stats(nullptr, nullptr, &st) == BPSF_EINVAL);
  EXPECT(bpsf_bp_trace(nullptr, u8, d8, &q, nullptr, nullptr, u8, i32, u8) == BPSF_EINVAL);
  EXPECT(bpsf_set_timing(nullptr, 1) == BPSF_EINVAL);
  EXPECT(bpsf_last_timing(nullptr, f4) == BPSF_EINVAL);
  EXPECT(bpsf_tile_options(nullptr, i32, 8) == BPSF_EINVAL);
  EXPECT(bpsf_set_tile(nullptr, 1, 1) == BPSF_EINVAL);
  bpsf_tuning tu;
  EXPECT(bpsf_autotune(nullptr, u8, d8, 1, &q, 1, nullptr, &tu) == BPSF_EINVAL);
  EXPECT(bpsf_set_trial_table(nullptr, nullptr, 0, 0) == BPSF_EINVAL);
  EXPECT(bpsf_set_trial_table64(nullptr, nullptr, 0, 0) == BPSF_EINVAL);
  EXPECT(bpsf_code_info(nullptr, i32, i32, i32, i32, i32) == BPSF_EINVAL);
  bpsf_free_code(nullptr);
  bpsf_mix mx = nullptr;
  EXPECT(bpsf_mix_create(nullptr, 1, &mx) == BPSF_EINVAL);
  bpsf_code none[2] = {nullptr, nullptr};
  EXPECT(bpsf_mix_create(none, 2, &mx) == BPSF_EINVAL);
  EXPECT(bpsf_mix_create(none, 0, &mx) == BPSF_EINVAL);
  EXPECT(bpsf_mix_create(none, 9, &mx) == BPSF_EINVAL);
  const double* pr[1] = {d8};
  EXPECT(bpsf_mix_decode(nullptr, i32, u8, 8, pr, 1, &q, u8, 8, u8, i32, nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_mix_decode_grouped(nullptr, i64, u8, 8, pr, &q, u8, 8, u8, i32, nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_mix_reserve(nullptr, 10, &q) == BPSF_EINVAL);
  EXPECT(bpsf_mix_last_stats(nullptr, nullptr, &st, i64) == BPSF_EINVAL);
  bpsf_mix_free(nullptr);
  bpsf_server sv = nullptr;
  EXPECT(bpsf_server_create(nullptr, 1, pr, &q, 1, 16, 1, 0, &sv) == BPSF_EINVAL);
  EXPECT(bpsf_server_create(none, 1, pr, &q, 0, 16, 1, 0, &sv) == BPSF_EINVAL);
  EXPECT(bpsf_server_create(none, 1, pr, &q, 2, 16, 0, 0, &sv) == BPSF_EINVAL);
  EXPECT(bpsf_server_create(none, 1, pr, &q, 1, 0, 1, 0, &sv) == BPSF_EINVAL);
  EXPECT(bpsf_server_create(none, 1, pr, &q, 1, 16, 1, -5, &sv) == BPSF_EINVAL);
  EXPECT(bpsf_server_create(none, 1, pr, &q, 1, 16, 1, 0, &sv) == BPSF_EINVAL);   // NULL code
  EXPECT(bpsf_server_submit(nullptr, 0, u8, 1, u8, u8, i32, i64) == BPSF_EINVAL);
  EXPECT(bpsf_server_wait(nullptr, 1, nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_server_poll(nullptr, i64, 4) == BPSF_EINVAL);
  EXPECT(bpsf_server_replay(nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr) == BPSF_EINVAL);
  EXPECT(bpsf_server_counters(nullptr, i64, i64, i64) == BPSF_EINVAL);
  EXPECT(bpsf_server_memory(nullptr, i64, i64, i64, i64, i64) == BPSF_EINVAL);
  EXPECT(bpsf_server_destroy(nullptr) == 0);
  if (fails) return 1;
  printf("runtime sanitizer driver: ok\n");
  return 0;
}
