// Request loop of the BP-SF library (bpsf_server_*; C ABI in include/bpsf.h).
//
// Requests are batches of host syndromes of one code of a mix. A worker
// thread owns L "lanes", each with its own stream, its own mix handle and
// pinned host staging; device memory comes from one pool per server whose
// size is the caller's budget or half the device memory free at creation.
// Whenever a lane is free and requests are waiting, the worker admits, in
// arrival order, as many waiting requests as fit the batch limit and a free
// region of the pool (their syndromes, outputs and decode scratch), copies
// them to the device grouped by code, decodes them with one mixed decode
// (one persistent launch per phase over all codes of the batch, its scratch
// in the region) and copies the results back in one transfer; requests that
// do not fit wait until a batch ends and returns its region. While a batch
// runs, later arrivals queue up for the next free lane, so work of several
// batches overlaps on the device. Completed lanes are found by querying their
// events; their results are scattered to the requests' host buffers. Every
// kernel shape the server can launch is run once at creation.
//
// In per-request mode the worker instead decodes each request by itself with
// bpsf_decode on its code, in arrival order on one lane: the plain
// one-launch-sequence-per-request form the batched mode is measured against.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bpsf.h"
#include "bpsf_internal.h"

namespace {

int sfail(int code, const char* fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return bpsf::report_error(code, buf);
}

double now_s()
{
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  int code = 0;
  int n = 0;
  const uint8_t* syn = nullptr;
  uint8_t* corr = nullptr;
  uint8_t* conv = nullptr;
  int32_t* it = nullptr;
  double t_submit = 0.0, t_done = 0.0;
  int64_t row = 0;          // first row of the request in its lane's batch
  bool done = false;
  bool waited = false;      // waited for device memory at least once
  int rc = 0;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bpsf_mix mix = nullptr;
  uint8_t* h_syn = nullptr;   // pinned: cap rows of mmax bytes
  uint8_t* h_out = nullptr;   // pinned: the output block of a batch of cap shots
  size_t off = 0, len = 0;    // the batch's region of the device pool
  size_t in_stride = 0, out_stride = 0;   // row bytes of the batch's syndromes and corrections
  std::vector<Request*> reqs;
  int64_t shots = 0;
  bool busy = false;        // taken by the worker (from admission until the batch is retired)
  bool in_flight = false;   // launched: the completion thread polls its event
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// A batch of n shots in the device pool: syndromes, then one output block
// (corrections [n][nmax], converged [n], iterations [n], each 256-aligned, so
// one copy brings them back), then the decode's scratch.
struct BatchLayout {
  size_t syn, out, conv, it, out_bytes, scratch, total;
};

// First-fit allocator over the server's device pool (offsets, 256-byte units).
struct Pool {
  unsigned char* base = nullptr;
  size_t bytes = 0, in_use = 0, peak = 0;
  std::map<size_t, size_t> free_;   // offset -> length, neighbours merged

  void init(void* b, size_t n)
  {
    base = static_cast<unsigned char*>(b);
    bytes = n;
    free_.clear();
    free_[0] = n;
  }
  bool take(size_t want, size_t* off)
  {
    want = al256(want);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < want) continue;
      *off = it->first;
      const size_t rest = it->second - want;
      const size_t at = it->first + want;
      free_.erase(it);
      if (rest) free_[at] = rest;
      in_use += want;
      peak = std::max(peak, in_use);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t len)
  {
    len = al256(len);
    in_use -= len;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct bpsf_server_s {
  int device = 0;
  int n_codes = 0;
  bpsf_code codes[8] = {};
  int M[8] = {}, N[8] = {};
  int mmax = 0, nmax = 0;
  std::vector<std::vector<double>> priors;
  const double* prior_ptr[8] = {};
  bpsf_params params{};
  int batching = 1;
  int64_t cap = 0;            // shots per batch at most (the caller's limit)
  int64_t max_request = 0;    // the largest request the pool can ever hold (<= cap)
  int scratch_stride = 0;     // record words per shot of a batch's decode scratch
  size_t keep_bytes = 0;      // room per batch for kept trial corrections (batched mode)
  void* pool_mem = nullptr;
  Pool pool;
  std::vector<Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_busy;
  std::deque<Request*> pending;
  std::unordered_map<int64_t, Request*> live;
  std::deque<int64_t> completed;
  int64_t next_id = 1;
  bool stop = false;
  bool worker_done = false;
  int worker_rc = 0;
  std::thread worker, completer;
  // counters
  int64_t batches = 0, batch_shots = 0, requests_done = 0, waited_for_memory = 0;
};

namespace {

BatchLayout layout_of(const bpsf_server_s* s, int64_t n, size_t scratch)
{
  BatchLayout L;
  const size_t k = (size_t)n;
  L.syn = 0;
  L.out = al256(k * s->mmax);
  L.conv = L.out + al256(k * s->nmax);
  L.it = L.conv + al256(k);
  L.out_bytes = L.it - L.out + 4 * k;
  L.scratch = al256(L.it + 4 * k);
  L.total = L.scratch + scratch;
  return L;
}

// Room a batched-mode batch adds to its scratch for the corrections that its
// trials keep (the last phase then copies the winners' instead of decoding
// them again; 1 MiB keeps about 130 records of a 64-trial small-family decode
// of one code, a fifth of that with five codes in the batch: every failed
// shot of a small batch): at most a sixteenth of a caller's device budget.
constexpr size_t KEEP_BYTES = (size_t)1 << 20;

// The device bytes of a batch of n shots (its scratch: the mixed decode's,
// and room for kept trial corrections, in batched mode; per-request decodes
// use their code's own scratch).
int batch_layout(bpsf_server_s* s, int64_t n, BatchLayout* out)
{
  const size_t scratch =
      s->batching ? bpsf::mix_scratch_size(s->n_codes, n, s->scratch_stride) + s->keep_bytes : 0;
  *out = layout_of(s, n, scratch);
  return 0;
}

int lane_alloc(bpsf_server_s* s, Lane& l)
{
  const size_t cap = (size_t)s->cap;
  if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess)
    return sfail(BPSF_EDEVICE, "stream or event creation failed");
  const BatchLayout L = layout_of(s, s->cap, 0);
  if (hipHostMalloc((void**)&l.h_syn, cap * s->mmax, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&l.h_out, L.out_bytes, hipHostMallocDefault) != hipSuccess)
    return sfail(BPSF_ENOMEM, "pinned staging of a lane (%zu shots)", cap);
  if (s->batching) {
    const int rc = bpsf_mix_create(s->codes, s->n_codes, &l.mix);
    if (rc) return sfail(rc, "mix for a lane: %s", bpsf_last_error());
  } else {
    for (int c = 0; c < s->n_codes; ++c) {
      const int rc = bpsf_reserve(s->codes[c], s->cap, &s->params);
      if (rc) return sfail(rc, "scratch of code %d: %s", c, bpsf_last_error());
    }
  }
  return 0;
}

void lane_free(Lane& l)
{
  if (l.stream) (void)hipStreamSynchronize(l.stream);
  if (l.mix) bpsf_mix_free(l.mix);
  for (void* p : {(void*)l.h_syn, (void*)l.h_out})
    if (p) (void)hipHostFree(p);
  if (l.done) (void)hipEventDestroy(l.done);
  if (l.stream) (void)hipStreamDestroy(l.stream);
  l = Lane();
}

// Enqueue a batch on the lane: copy in, decode, one copy out, record. The
// lane's region (l.off, l.len) holds layout L; counts: shots per code, the
// staged rows grouped by code. A batch of one code has rows of that code's M
// and N bytes and takes the single-code call (per-request mode: bpsf_decode
// itself; batched mode: the same with its scratch in the region, which
// spares a lone request the mixed call's host work over every code); a
// batch of several codes has rows of the largest M and N.
int enqueue(bpsf_server_s* s, Lane& l, const int64_t* counts, int64_t n, const BatchLayout& L)
{
  unsigned char* d = s->pool.base + l.off;
  if (hipMemcpyAsync(d + L.syn, l.h_syn, (size_t)n * l.in_stride, hipMemcpyHostToDevice, l.stream) != hipSuccess)
    return sfail(BPSF_EDEVICE, "copy in");
  uint8_t* corr = d + L.out;
  uint8_t* conv = d + L.conv;
  int32_t* it = reinterpret_cast<int32_t*>(d + L.it);
  int present = 0, only = 0;
  for (int c = 0; c < s->n_codes; ++c)
    if (counts[c] > 0) {
      ++present;
      only = c;
    }
  int rc = 0;
  if (present == 1 && !s->batching) {
    rc = bpsf_decode(s->codes[only], d + L.syn, s->prior_ptr[only], n, &s->params, corr, conv, it, l.stream);
  } else if (present == 1) {
    rc = bpsf::decode_in(s->codes[only], d + L.syn, s->prior_ptr[only], n, &s->params, corr, conv, it, l.stream,
                         d + L.scratch, L.total - L.scratch);
  } else {
    rc = bpsf::mix_decode_grouped_in(l.mix, counts, d + L.syn, (int64_t)l.in_stride, s->prior_ptr, &s->params, corr,
                                     (int64_t)l.out_stride, conv, it, l.stream, d + L.scratch, L.total - L.scratch);
  }
  if (rc) return sfail(rc, "decode: %s", bpsf_last_error());
  if (hipMemcpyAsync(l.h_out, d + L.out, L.out_bytes, hipMemcpyDeviceToHost, l.stream) != hipSuccess ||
      hipEventRecord(l.done, l.stream) != hipSuccess)
    return sfail(BPSF_EDEVICE, "copy out");
  return 0;
}

// Row strides of a batch: a code's own M and N when the batch holds one code,
// else the largest.
void set_strides(const bpsf_server_s* s, Lane& l, const int64_t* counts)
{
  int present = 0, only = 0;
  for (int c = 0; c < s->n_codes; ++c)
    if (counts[c] > 0) {
      ++present;
      only = c;
    }
  l.in_stride = present == 1 ? (size_t)s->M[only] : (size_t)s->mmax;
  l.out_stride = present == 1 ? (size_t)s->N[only] : (size_t)s->nmax;
}

// Stage and enqueue the lane's requests (rows grouped by code).
int lane_launch(bpsf_server_s* s, Lane& l, const BatchLayout& L)
{
  int64_t counts[8] = {}, next[8] = {};
  for (Request* r : l.reqs) counts[r->code] += r->n;
  for (int c = 1; c < s->n_codes; ++c) next[c] = next[c - 1] + counts[c - 1];
  set_strides(s, l, counts);
  const size_t stride = l.in_stride;
  for (Request* r : l.reqs) {
    const int m = s->M[r->code];
    r->row = next[r->code];
    next[r->code] += r->n;
    if (stride == (size_t)m) {
      memcpy(l.h_syn + (size_t)r->row * stride, r->syn, (size_t)r->n * m);
    } else {
      for (int i = 0; i < r->n; ++i) memcpy(l.h_syn + (size_t)(r->row + i) * stride, r->syn + (size_t)i * m, (size_t)m);
    }
  }
  return enqueue(s, l, counts, l.shots, L);
}

// Scatter a finished lane's results to its requests (worker thread, no lock held).
void lane_scatter(bpsf_server_s* s, Lane& l)
{
  const BatchLayout L = layout_of(s, l.shots, 0);
  const uint8_t* corr = l.h_out;
  const uint8_t* conv = l.h_out + (L.conv - L.out);
  const int32_t* it = reinterpret_cast<const int32_t*>(l.h_out + (L.it - L.out));
  for (Request* r : l.reqs) {
    const int nb = s->N[r->code];
    const size_t stride = l.out_stride;
    if (stride == (size_t)nb) {
      memcpy(r->corr, corr + (size_t)r->row * stride, (size_t)r->n * nb);
    } else {
      for (int i = 0; i < r->n; ++i) memcpy(r->corr + (size_t)i * nb, corr + (size_t)(r->row + i) * stride, (size_t)nb);
    }
    memcpy(r->conv, conv + r->row, (size_t)r->n);
    memcpy(r->it, it + r->row, 4 * (size_t)r->n);
  }
}

// Decodes of zero syndromes in every shape the server's batches can take
// (each code alone and all codes together, one shot each and the largest
// batch), so that every kernel is loaded and every launch shape queried
// before the first request: a first use costs milliseconds.
int warm_up(bpsf_server_s* s)
{
  for (Lane& l : s->lanes) memset(l.h_syn, 0, (size_t)s->cap * s->mmax);
  std::vector<std::vector<int64_t>> shapes;
  for (int64_t n : {(int64_t)1, s->max_request}) {
    for (int c = 0; c < s->n_codes; ++c) {
      std::vector<int64_t> v((size_t)s->n_codes, 0);
      v[(size_t)c] = n;
      shapes.push_back(v);
    }
    if (s->batching && s->n_codes > 1) {
      std::vector<int64_t> v((size_t)s->n_codes, std::max<int64_t>(1, n / s->n_codes));
      shapes.push_back(v);
    }
  }
  // every shape on the first lane, one after the other
  auto run = [&](Lane& l, const std::vector<int64_t>& v) {
    int64_t n = 0;
    for (int64_t x : v) n += x;
    BatchLayout L;
    int rc = batch_layout(s, n, &L);
    if (rc) return rc;
    if (!s->pool.take(L.total, &l.off)) return sfail(BPSF_ENOMEM, "warm-up batch of %lld shots", (long long)n);
    l.len = L.total;
    set_strides(s, l, v.data());
    rc = enqueue(s, l, v.data(), n, L);
    if (rc) s->pool.give(l.off, l.len);
    return rc;
  };
  auto drain = [&](Lane& l) {
    const int rc = hipStreamSynchronize(l.stream) == hipSuccess ? 0 : sfail(BPSF_EDEVICE, "warm-up");
    s->pool.give(l.off, l.len);
    return rc;
  };
  int rc = 0;
  for (const auto& v : shapes) {
    if ((rc = run(s->lanes[0], v))) return rc;
    if ((rc = drain(s->lanes[0]))) return rc;
  }
  // Then every lane at once, twice: the copies of requests of every size
  // class (each code's rows and the widest rows, 1..16 shots and powers of
  // two), and decodes of one shot and of up to 256 shots. The runtime sets up
  // a copy path the first time a stream uses it, and differently when other
  // streams have work in flight: a first device-to-host copy of a 75-shot
  // batch while the other lane ran measured 6.7 ms on the host.
  int64_t per_lane = 0;   // the largest batch a lane's share of the pool holds
  {
    int64_t lo = 0, hi = s->max_request;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      BatchLayout L;
      if ((rc = batch_layout(s, mid, &L))) return rc;
      if (al256(L.total) * s->lanes.size() <= s->pool.bytes) lo = mid;
      else hi = mid - 1;
    }
    per_lane = lo;
  }
  if (per_lane < 1) {
    s->pool.peak = 0;
    return 0;   // lanes never run at once in a pool this small
  }
  std::vector<int64_t> ns;
  for (int64_t n = 1; n <= std::min<int64_t>(16, per_lane); ++n) ns.push_back(n);
  for (int64_t n = 32; n < per_lane; n *= 2) ns.push_back(n);
  ns.push_back(per_lane);
  for (int rep = 0; rep < 2 && !rc; ++rep) {
    std::vector<Lane*> holding;
    for (Lane& l : s->lanes) {
      BatchLayout L;
      if ((rc = batch_layout(s, per_lane, &L))) break;
      if (!s->pool.take(L.total, &l.off)) {
        rc = sfail(BPSF_ENOMEM, "warm-up copies");
        break;
      }
      l.len = L.total;
      holding.push_back(&l);
      unsigned char* d = s->pool.base + l.off;
      for (int c = 0; c <= s->n_codes && !rc; ++c) {
        const size_t m = c < s->n_codes ? (size_t)s->M[c] : (size_t)s->mmax;
        for (int64_t n : ns) {
          // (the output block's size depends only on the shot count)
          if (hipMemcpyAsync(d + L.syn, l.h_syn, (size_t)n * m, hipMemcpyHostToDevice, l.stream) != hipSuccess ||
              hipMemcpyAsync(l.h_out, d + L.out, layout_of(s, n, 0).out_bytes, hipMemcpyDeviceToHost, l.stream) !=
                  hipSuccess) {
            rc = sfail(BPSF_EDEVICE, "warm-up copy");
            break;
          }
        }
      }
      if (rc) break;
    }
    for (Lane* l : holding) {
      const int r2 = drain(*l);
      if (!rc) rc = r2;
    }
  }
  if (rc) return rc;
  std::vector<std::vector<int64_t>> together;
  for (int64_t n : {(int64_t)1, std::min<int64_t>(256, per_lane)}) {
    std::vector<int64_t> v((size_t)s->n_codes, 0);
    v[0] = n;
    together.push_back(v);
    if (s->batching && s->n_codes > 1) {
      std::vector<int64_t> w((size_t)s->n_codes, std::max<int64_t>(1, n / s->n_codes));
      together.push_back(w);
    }
  }
  for (int rep = 0; rep < 2; ++rep) {
    for (const auto& v : together) {
      size_t started = 0;
      for (; started < s->lanes.size() && !rc; ++started) rc = run(s->lanes[started], v);
      if (rc) --started;
      for (size_t i = 0; i < started; ++i) {
        const int r2 = drain(s->lanes[i]);
        if (!rc) rc = r2;
      }
      if (rc) return rc;
    }
  }
  s->pool.peak = 0;
  return 0;
}

// Completion thread: finds finished batches by querying their lanes'
// events, scatters their results (no lock held), then marks the requests done
// and returns the lanes and their pool regions. Launching is the worker's:
// a completion is never held up behind another lane's launch.
void completer_main(bpsf_server_s* s)
{
  (void)hipSetDevice(s->device);
  // short timed waits wake on time (the default 50 us slack would add to
  // every request's latency)
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::vector<Lane*> busy;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    busy.clear();
    for (Lane& l : s->lanes)
      if (l.in_flight) busy.push_back(&l);
    if (busy.empty()) {
      if (s->worker_done) break;
      s->cv_busy.wait(lk);
      continue;
    }
    lk.unlock();
    bool any = false;
    for (Lane* l : busy) {
      const hipError_t q = hipEventQuery(l->done);
      if (q == hipErrorNotReady) continue;
      if (q == hipSuccess) lane_scatter(s, *l);
      const double t = now_s();
      lk.lock();
      for (Request* r : l->reqs) {
        r->t_done = t;
        r->done = true;
        r->rc = q == hipSuccess ? 0 : BPSF_EDEVICE;
        s->completed.push_back(r->id);
        ++s->requests_done;
      }
      if (q != hipSuccess && !s->worker_rc) s->worker_rc = BPSF_EDEVICE;
      s->pool.give(l->off, l->len);
      l->reqs.clear();
      l->shots = 0;
      l->in_flight = false;
      l->busy = false;
      lk.unlock();
      s->cv_done.notify_all();
      s->cv_work.notify_one();
      any = true;
    }
    lk.lock();
    // poll the device again shortly (a launch wakes us at once)
    if (!any) s->cv_busy.wait_for(lk, std::chrono::microseconds(5));
  }
}

// Admission and launch thread: whenever a lane is free and requests wait, it
// admits, in arrival order, as many as fit the batch limit and a free region
// of the device pool, and launches them; the rest wait for a lane or for
// memory to come back (a completion wakes it).
void worker_main(bpsf_server_s* s)
{
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool launched = false, blocked = false;
    for (Lane& l : s->lanes) {
      if (l.busy || s->pending.empty()) continue;
      int64_t take = 0, shots = 0;
      if (s->batching) {
        for (Request* r : s->pending) {
          if (shots + r->n > s->cap) break;
          shots += r->n;
          ++take;
        }
      } else {
        take = 1;
        shots = s->pending.front()->n;
      }
      BatchLayout L;
      int rc = 0;
      bool fits = false;
      while (take > 0) {
        if ((rc = batch_layout(s, shots, &L))) break;
        if ((fits = s->pool.take(L.total, &l.off))) break;
        shots -= s->pending[(size_t)take - 1]->n;
        --take;
      }
      if (!rc && !fits) {
        // not even the first request fits now: it waits for a batch to end
        Request* r = s->pending.front();
        if (!r->waited) {
          r->waited = true;
          ++s->waited_for_memory;
        }
        blocked = true;
        break;
      }
      l.len = rc ? 0 : L.total;
      l.reqs.assign(s->pending.begin(), s->pending.begin() + take);
      s->pending.erase(s->pending.begin(), s->pending.begin() + take);
      l.shots = shots;
      l.busy = true;   // owned by this thread until launched
      if (!rc) {
        lk.unlock();
        rc = lane_launch(s, l, L);
        lk.lock();
      }
      if (rc) {
        if (l.len) s->pool.give(l.off, l.len);
        for (Request* r : l.reqs) {
          r->done = true;
          r->rc = rc;
          s->completed.push_back(r->id);
        }
        l.reqs.clear();
        l.busy = false;
        s->worker_rc = rc;
        s->cv_done.notify_all();
        continue;
      }
      l.in_flight = true;
      launched = true;
      ++s->batches;
      s->batch_shots += l.shots;
      s->cv_busy.notify_one();
    }
    if (s->stop && s->pending.empty()) break;
    if (launched) continue;
    // wait for a submission, a lane or pool memory coming back, or stop
    bool free_lane = false;
    for (Lane& l : s->lanes) free_lane = free_lane || !l.busy;
    if (!s->pending.empty() && free_lane && !blocked) continue;
    s->cv_work.wait(lk);
  }
  s->worker_done = true;
  s->cv_busy.notify_all();
}

}  // namespace

extern "C" {

int bpsf_server_create(const bpsf_code* codes, int32_t n_codes, const double* const* priors,
                       const bpsf_params* params, int32_t lanes, int64_t max_batch_shots, int32_t batching,
                       int64_t device_budget_bytes, bpsf_server* out)
{
  if (!out) return sfail(BPSF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!codes || n_codes < 1 || n_codes > 8 || !priors || !params)
    return sfail(BPSF_EINVAL, "need 1..8 codes, their priors and params");
  if (lanes < 1 || lanes > 8) return sfail(BPSF_EINVAL, "lanes must be in 1..8");
  if (!batching && lanes != 1) return sfail(BPSF_EINVAL, "per-request mode runs one lane");
  if (max_batch_shots < 1 || max_batch_shots > (1 << 24)) return sfail(BPSF_EINVAL, "max_batch_shots in 1..2^24");
  if (device_budget_bytes < 0) return sfail(BPSF_EINVAL, "device_budget_bytes < 0");
  if (params->flags & BPSF_FLAG_LAYERED) return sfail(BPSF_ENOTSUP, "the server runs the flooding schedule only");
  if (params->k > 16) return sfail(BPSF_ENOTSUP, "the server takes |Phi| up to 16");
  bpsf_server_s* s = new (std::nothrow) bpsf_server_s;
  if (!s) return sfail(BPSF_ENOMEM, "handle");
  (void)hipGetDevice(&s->device);
  s->n_codes = n_codes;
  s->params = *params;
  s->batching = batching != 0;
  s->cap = max_batch_shots;
  s->priors.resize(n_codes);
  for (int c = 0; c < n_codes; ++c) {
    s->codes[c] = codes[c];
    int32_t M = 0, N = 0;
    if (!codes[c] || bpsf_code_info(codes[c], &M, &N, nullptr, nullptr, nullptr)) {
      delete s;
      return sfail(BPSF_EINVAL, "codes[%d] is not a loaded code", c);
    }
    s->M[c] = M;
    s->N[c] = N;
    s->mmax = std::max(s->mmax, (int)M);
    s->nmax = std::max(s->nmax, (int)N);
    if (!priors[c]) {
      delete s;
      return sfail(BPSF_EINVAL, "priors[%d] is NULL", c);
    }
    s->priors[c].assign(priors[c], priors[c] + N);
    s->prior_ptr[c] = s->priors[c].data();
  }
  s->lanes.resize(lanes);
  int rc = 0;
  for (Lane& l : s->lanes)
    if ((rc = lane_alloc(s, l))) break;
  // the device pool: the caller's budget, or half the device memory free now
  // (no more than every lane holding a full batch)
  if (!rc && s->batching) {
    rc = bpsf::mix_scratch_stride(s->lanes[0].mix, &s->params, &s->scratch_stride);
    if (rc) rc = sfail(rc, "scratch of a batch: %s", bpsf_last_error());
  }
  s->keep_bytes = device_budget_bytes > 0 ? std::min(KEEP_BYTES, al256((size_t)device_budget_bytes / 16)) : KEEP_BYTES;
  BatchLayout full;
  if (!rc) rc = batch_layout(s, s->cap, &full);
  size_t budget = 0;
  if (!rc) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      rc = sfail(BPSF_EDEVICE, "hipMemGetInfo");
    } else if (device_budget_bytes > 0) {
      budget = al256((size_t)device_budget_bytes);
      if (budget > free_b) rc = sfail(BPSF_ENOMEM, "a budget of %zu bytes exceeds the %zu bytes free", budget, free_b);
    } else {
      budget = std::min(al256(free_b / 2), al256(full.total) * (size_t)lanes);
    }
  }
  // the largest request the whole pool can hold
  if (!rc) {
    int64_t lo = 0, hi = s->cap;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      BatchLayout L;
      if ((rc = batch_layout(s, mid, &L))) break;
      if (al256(L.total) <= budget) lo = mid;
      else hi = mid - 1;
    }
    s->max_request = lo;
    if (!rc && lo < 1) rc = sfail(BPSF_EINVAL, "a device budget of %zu bytes holds no batch", budget);
  }
  if (!rc && hipMalloc(&s->pool_mem, budget) != hipSuccess) rc = sfail(BPSF_ENOMEM, "device pool of %zu bytes", budget);
  if (!rc) {
    s->pool.init(s->pool_mem, budget);
    rc = warm_up(s);
  }
  if (rc) {
    for (Lane& l : s->lanes) lane_free(l);
    if (s->pool_mem) (void)hipFree(s->pool_mem);
    delete s;
    return rc;
  }
  s->worker = std::thread(worker_main, s);
  s->completer = std::thread(completer_main, s);
  *out = s;
  return 0;
}

int bpsf_server_submit(bpsf_server s, int32_t code, const uint8_t* syndromes, int32_t n, uint8_t* corrections,
                       uint8_t* converged, int32_t* iterations, int64_t* id_out)
{
  if (!s || !id_out) return sfail(BPSF_EINVAL, "NULL argument");
  if (code < 0 || code >= s->n_codes) return sfail(BPSF_EINVAL, "code %d out of range", code);
  if (n < 1 || n > s->max_request)
    return sfail(BPSF_EINVAL, "a request holds 1..%lld shots (batch limit %lld, device budget %zu bytes)",
                 (long long)s->max_request, (long long)s->cap, s->pool.bytes);
  if (!syndromes || !corrections || !converged || !iterations) return sfail(BPSF_EINVAL, "NULL buffer");
  Request* r = new (std::nothrow) Request;
  if (!r) return sfail(BPSF_ENOMEM, "request");
  r->code = code;
  r->n = n;
  r->syn = syndromes;
  r->corr = corrections;
  r->conv = converged;
  r->it = iterations;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return sfail(BPSF_EINVAL, "server is stopping");
    }
    r->id = s->next_id++;
    s->live[r->id] = r;
    s->pending.push_back(r);
  }
  s->cv_work.notify_one();
  *id_out = r->id;
  return 0;
}

int bpsf_server_wait(bpsf_server s, int64_t id, double* latency_s_out)
{
  if (!s) return sfail(BPSF_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto itr = s->live.find(id);
  if (itr == s->live.end()) return sfail(BPSF_EINVAL, "unknown or already collected request %lld", (long long)id);
  Request* r = itr->second;
  s->cv_done.wait(lk, [r] { return r->done; });
  const int rc = r->rc;
  if (latency_s_out) *latency_s_out = r->t_done - r->t_submit;
  s->live.erase(itr);
  delete r;
  return rc ? sfail(rc, "request failed on the device") : 0;
}

int64_t bpsf_server_poll(bpsf_server s, int64_t* ids_out, int64_t cap)
{
  if (!s || (!ids_out && cap > 0)) return sfail(BPSF_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int64_t n = 0;
  while (n < cap && !s->completed.empty()) {
    ids_out[n++] = s->completed.front();
    s->completed.pop_front();
  }
  return n;
}

int bpsf_server_replay(bpsf_server s, int64_t n_req, const double* arrival_s, const int32_t* code,
                       const int32_t* shots, const uint8_t* const* syndromes, uint8_t* const* corrections,
                       uint8_t* const* converged, int32_t* const* iterations, double* latency_s,
                       double* wall_s)
{
  if (!s || n_req < 0 || (n_req > 0 && (!arrival_s || !code || !shots || !syndromes || !corrections ||
                                        !converged || !iterations || !latency_s)))
    return sfail(BPSF_EINVAL, "NULL argument");
  std::vector<int64_t> ids((size_t)n_req);
  std::vector<double> due((size_t)n_req);
  const double t0 = now_s();
  int rc = 0;
  for (int64_t i = 0; i < n_req && !rc; ++i) {
    due[i] = t0 + arrival_s[i];
    // open loop: submit at the scheduled time whatever is still in flight
    for (;;) {
      const double left = due[i] - now_s();
      if (left <= 0) break;
      if (left > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(left - 1e-4));
    }
    rc = bpsf_server_submit(s, code[i], syndromes[i], shots[i], corrections[i], converged[i], iterations[i], &ids[i]);
    if (rc) n_req = i;
  }
  for (int64_t i = 0; i < n_req; ++i) {
    std::unique_lock<std::mutex> lk(s->mu);
    auto itr = s->live.find(ids[i]);
    if (itr == s->live.end()) continue;
    Request* r = itr->second;
    s->cv_done.wait(lk, [r] { return r->done; });
    latency_s[i] = r->t_done - due[i];
    if (r->rc && !rc) rc = sfail(r->rc, "request failed on the device");
    s->live.erase(itr);
    delete r;
  }
  if (wall_s) *wall_s = now_s() - t0;
  // drop completion notices of the replayed requests
  std::lock_guard<std::mutex> lk(s->mu);
  s->completed.clear();
  return rc;
}

int bpsf_server_counters(bpsf_server s, int64_t* batches, int64_t* batch_shots, int64_t* requests_done)
{
  if (!s) return sfail(BPSF_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (batches) *batches = s->batches;
  if (batch_shots) *batch_shots = s->batch_shots;
  if (requests_done) *requests_done = s->requests_done;
  return 0;
}

int bpsf_server_memory(bpsf_server s, int64_t* budget, int64_t* in_use, int64_t* peak, int64_t* max_request,
                       int64_t* waited_for_memory)
{
  if (!s) return sfail(BPSF_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (budget) *budget = (int64_t)s->pool.bytes;
  if (in_use) *in_use = (int64_t)s->pool.in_use;
  if (peak) *peak = (int64_t)s->pool.peak;
  if (max_request) *max_request = s->max_request;
  if (waited_for_memory) *waited_for_memory = s->waited_for_memory;
  return 0;
}

int bpsf_server_destroy(bpsf_server s)
{
  if (!s) return 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->completer.joinable()) s->completer.join();
  for (Lane& l : s->lanes) lane_free(l);
  if (s->pool_mem) (void)hipFree(s->pool_mem);
  for (auto& kv : s->live) delete kv.second;
  const int rc = s->worker_rc;
  delete s;
  return rc;
}

}  // extern "C"
