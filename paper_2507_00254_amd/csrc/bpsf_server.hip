// Request loop of the BP-SF library (bpsf_server_*; C ABI in include/bpsf.h).
//
// Requests are batches of host syndromes of one code of a mix. A worker
// thread owns L "lanes", each with its own stream, its own mix handle (so
// its scratch is private), device buffers for `cap` shots and pinned host
// staging. Whenever a lane is free and requests are waiting, the worker packs
// every waiting request that fits the lane's budget into one batch, copies it
// to the device grouped by code, decodes it with one bpsf_mix_decode_grouped
// (one persistent launch
// per phase over all codes of the batch) and copies the results back; while
// that runs, later arrivals queue up for the next free lane, so work of
// several batches overlaps on the device. Completed lanes are found by
// querying their events; their results are scattered to the requests' host
// buffers.
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
  int rc = 0;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bpsf_mix mix = nullptr;
  void *d_syn = nullptr, *d_corr = nullptr, *d_conv = nullptr, *d_it = nullptr;
  uint8_t *h_syn = nullptr, *h_corr = nullptr, *h_conv = nullptr;
  int32_t* h_it = nullptr;
  std::vector<Request*> reqs;
  int64_t shots = 0;
  bool busy = false;
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
  int64_t cap = 0;
  std::vector<Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<int64_t, Request*> live;
  std::deque<int64_t> completed;
  int64_t next_id = 1;
  bool stop = false;
  int worker_rc = 0;
  std::thread worker;
  // counters
  int64_t batches = 0, batch_shots = 0, requests_done = 0;
};

namespace {

int lane_alloc(bpsf_server_s* s, Lane& l)
{
  const size_t cap = (size_t)s->cap;
  if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess)
    return sfail(BPSF_EDEVICE, "stream or event creation failed");
  if (hipMalloc(&l.d_syn, cap * s->mmax) != hipSuccess ||
      hipMalloc(&l.d_corr, cap * s->nmax) != hipSuccess || hipMalloc(&l.d_conv, cap) != hipSuccess ||
      hipMalloc(&l.d_it, 4 * cap) != hipSuccess)
    return sfail(BPSF_ENOMEM, "device buffers of a lane (%zu shots)", cap);
  if (hipHostMalloc((void**)&l.h_syn, cap * s->mmax, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&l.h_corr, cap * s->nmax, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&l.h_conv, cap, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&l.h_it, 4 * cap, hipHostMallocDefault) != hipSuccess)
    return sfail(BPSF_ENOMEM, "pinned staging of a lane (%zu shots)", cap);
  // scratch for a full batch now: no allocation (and no device-wide
  // synchronization it implies) once requests flow
  if (s->batching) {
    int rc = bpsf_mix_create(s->codes, s->n_codes, &l.mix);
    if (!rc) rc = bpsf_mix_reserve(l.mix, s->cap, &s->params);
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
  for (void* p : {l.d_syn, l.d_corr, l.d_conv, l.d_it})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)l.h_syn, (void*)l.h_corr, (void*)l.h_conv, (void*)l.h_it})
    if (p) (void)hipHostFree(p);
  if (l.done) (void)hipEventDestroy(l.done);
  if (l.stream) (void)hipStreamDestroy(l.stream);
  l = Lane();
}

// Enqueue the lane's batch: stage, copy in, decode, copy out, record.
int lane_launch(bpsf_server_s* s, Lane& l)
{
  const int64_t n = l.shots;
  if (s->batching) {
    // rows grouped by code, so the decode needs no device-side bucketing
    int64_t counts[8] = {}, next[8] = {};
    for (Request* r : l.reqs) counts[r->code] += r->n;
    for (int c = 1; c < s->n_codes; ++c) next[c] = next[c - 1] + counts[c - 1];
    for (Request* r : l.reqs) {
      const int m = s->M[r->code];
      r->row = next[r->code];
      next[r->code] += r->n;
      for (int i = 0; i < r->n; ++i)
        memcpy(l.h_syn + (size_t)(r->row + i) * s->mmax, r->syn + (size_t)i * m, (size_t)m);
    }
    if (hipMemcpyAsync(l.d_syn, l.h_syn, (size_t)n * s->mmax, hipMemcpyHostToDevice, l.stream) != hipSuccess)
      return sfail(BPSF_EDEVICE, "copy in");
    int rc = bpsf_mix_decode_grouped(l.mix, counts, static_cast<const uint8_t*>(l.d_syn), s->mmax, s->prior_ptr,
                                     &s->params, static_cast<uint8_t*>(l.d_corr), s->nmax,
                                     static_cast<uint8_t*>(l.d_conv), static_cast<int32_t*>(l.d_it), l.stream);
    if (rc) return sfail(rc, "mixed decode: %s", bpsf_last_error());
    if (hipMemcpyAsync(l.h_corr, l.d_corr, (size_t)n * s->nmax, hipMemcpyDeviceToHost, l.stream) != hipSuccess)
      return sfail(BPSF_EDEVICE, "copy out");
  } else {
    Request* r = l.reqs[0];
    const int m = s->M[r->code], nb = s->N[r->code];
    r->row = 0;
    memcpy(l.h_syn, r->syn, (size_t)r->n * m);
    if (hipMemcpyAsync(l.d_syn, l.h_syn, (size_t)r->n * m, hipMemcpyHostToDevice, l.stream) != hipSuccess)
      return sfail(BPSF_EDEVICE, "copy in");
    int rc = bpsf_decode(s->codes[r->code], static_cast<const uint8_t*>(l.d_syn), s->prior_ptr[r->code], r->n,
                         &s->params, static_cast<uint8_t*>(l.d_corr), static_cast<uint8_t*>(l.d_conv),
                         static_cast<int32_t*>(l.d_it), l.stream);
    if (rc) return sfail(rc, "decode: %s", bpsf_last_error());
    if (hipMemcpyAsync(l.h_corr, l.d_corr, (size_t)r->n * nb, hipMemcpyDeviceToHost, l.stream) != hipSuccess)
      return sfail(BPSF_EDEVICE, "copy out");
  }
  if (hipMemcpyAsync(l.h_conv, l.d_conv, (size_t)n, hipMemcpyDeviceToHost, l.stream) != hipSuccess ||
      hipMemcpyAsync(l.h_it, l.d_it, 4 * (size_t)n, hipMemcpyDeviceToHost, l.stream) != hipSuccess ||
      hipEventRecord(l.done, l.stream) != hipSuccess)
    return sfail(BPSF_EDEVICE, "copy out");
  return 0;
}

// Scatter a finished lane's results to its requests (worker thread, no lock held).
void lane_scatter(bpsf_server_s* s, Lane& l)
{
  for (Request* r : l.reqs) {
    const int nb = s->N[r->code];
    const size_t stride = s->batching ? (size_t)s->nmax : (size_t)nb;
    for (int i = 0; i < r->n; ++i) {
      const int64_t row = r->row + i;
      memcpy(r->corr + (size_t)i * nb, l.h_corr + (size_t)row * stride, (size_t)nb);
      r->conv[i] = l.h_conv[row];
      r->it[i] = l.h_it[row];
    }
  }
}

void worker_main(bpsf_server_s* s)
{
  (void)hipSetDevice(s->device);
  // short timed waits wake on time (the default 50 us slack would add to
  // every request's latency)
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // 1. finished lanes
    bool any_busy = false;
    for (Lane& l : s->lanes) {
      if (!l.busy) continue;
      const hipError_t q = hipEventQuery(l.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      lk.unlock();
      if (q == hipSuccess) lane_scatter(s, l);
      const double t = now_s();
      lk.lock();
      for (Request* r : l.reqs) {
        r->t_done = t;
        r->done = true;
        r->rc = q == hipSuccess ? 0 : BPSF_EDEVICE;
        s->completed.push_back(r->id);
        ++s->requests_done;
      }
      l.reqs.clear();
      l.shots = 0;
      l.busy = false;
      s->cv_done.notify_all();
    }
    // 2. admit waiting requests into free lanes
    bool launched = false;
    for (Lane& l : s->lanes) {
      if (l.busy || s->pending.empty()) continue;
      l.reqs.clear();
      l.shots = 0;
      if (s->batching) {
        while (!s->pending.empty() && l.shots + s->pending.front()->n <= s->cap) {
          l.reqs.push_back(s->pending.front());
          l.shots += s->pending.front()->n;
          s->pending.pop_front();
        }
      } else {
        l.reqs.push_back(s->pending.front());
        l.shots = s->pending.front()->n;
        s->pending.pop_front();
      }
      lk.unlock();
      const int rc = lane_launch(s, l);
      lk.lock();
      if (rc) {
        for (Request* r : l.reqs) {
          r->done = true;
          r->rc = rc;
          s->completed.push_back(r->id);
        }
        l.reqs.clear();
        s->worker_rc = rc;
        s->cv_done.notify_all();
        continue;
      }
      l.busy = true;
      any_busy = true;
      launched = true;
      ++s->batches;
      s->batch_shots += l.shots;
    }
    if (s->stop && s->pending.empty() && !any_busy) break;
    if (any_busy || launched) {
      // poll the device again shortly; new submissions wake us at once
      s->cv_work.wait_for(lk, std::chrono::microseconds(5));
    } else {
      s->cv_work.wait(lk, [s] { return s->stop || !s->pending.empty(); });
    }
  }
}

}  // namespace

extern "C" {

int bpsf_server_create(const bpsf_code* codes, int32_t n_codes, const double* const* priors,
                       const bpsf_params* params, int32_t lanes, int64_t max_batch_shots, int32_t batching,
                       bpsf_server* out)
{
  if (!out) return sfail(BPSF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!codes || n_codes < 1 || n_codes > 8 || !priors || !params)
    return sfail(BPSF_EINVAL, "need 1..8 codes, their priors and params");
  if (lanes < 1 || lanes > 8) return sfail(BPSF_EINVAL, "lanes must be in 1..8");
  if (!batching && lanes != 1) return sfail(BPSF_EINVAL, "per-request mode runs one lane");
  if (max_batch_shots < 1 || max_batch_shots > (1 << 24)) return sfail(BPSF_EINVAL, "max_batch_shots in 1..2^24");
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
  if (rc) {
    for (Lane& l : s->lanes) lane_free(l);
    delete s;
    return rc;
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return 0;
}

int bpsf_server_submit(bpsf_server s, int32_t code, const uint8_t* syndromes, int32_t n, uint8_t* corrections,
                       uint8_t* converged, int32_t* iterations, int64_t* id_out)
{
  if (!s || !id_out) return sfail(BPSF_EINVAL, "NULL argument");
  if (code < 0 || code >= s->n_codes) return sfail(BPSF_EINVAL, "code %d out of range", code);
  if (n < 1 || n > s->cap) return sfail(BPSF_EINVAL, "a request holds 1..%lld shots", (long long)s->cap);
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

int bpsf_server_destroy(bpsf_server s)
{
  if (!s) return 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Lane& l : s->lanes) lane_free(l);
  for (auto& kv : s->live) delete kv.second;
  const int rc = s->worker_rc;
  delete s;
  return rc;
}

}  // extern "C"
