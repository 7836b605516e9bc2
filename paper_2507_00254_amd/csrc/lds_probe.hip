// LDS bandwidth probe for gfx950: streaming ds_read / ds_write kernels whose
// measured rate is the peak the decoder's message traffic is compared with.
// C ABI declared in include/lds_probe.h; built as liblds_probe.so, apart from
// the decoder library.
//
// Every workgroup (four waves) owns 8 KB of LDS and its waves issue groups of
// eight LDS instructions of one kind in inline assembly, each group closed by
// one s_waitcnt inside the same asm statement (so no load is left in flight
// when the asm ends and nothing consumes the loaded registers: no VALU work
// competes with the LDS pipe). Lane l of a group touches bytes
// [l * B, (l + 1) * B) plus the group's offset, B the access width, which is
// the bank-conflict-free pattern for every width. Addresses stay inside the
// workgroup's 8 KB: widths 4/8/16 use lane bases below 1/2/4 KB and offsets
// below 8/4/2 steps of that size.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lds_probe.h"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_LDS_BYTES = 8192;
constexpr int PROBE_GROUP = 8;   // LDS instructions per asm statement

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(PROBE_THREADS) void probe_read_b32(int iters, uint32_t* out)
{
  const uint32_t a = threadIdx.x * 4u;   // < 1 KB; offsets up to 7 KB
  uint32_t r0, r1, r2, r3, r4, r5, r6, r7;
  for (int i = 0; i < iters; ++i) {
    asm volatile(
        "ds_read_b32 %0, %8\n"
        "ds_read_b32 %1, %8 offset:1024\n"
        "ds_read_b32 %2, %8 offset:2048\n"
        "ds_read_b32 %3, %8 offset:3072\n"
        "ds_read_b32 %4, %8 offset:4096\n"
        "ds_read_b32 %5, %8 offset:5120\n"
        "ds_read_b32 %6, %8 offset:6144\n"
        "ds_read_b32 %7, %8 offset:7168\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(a)
        : "memory");
  }
  if (iters < 0) out[threadIdx.x] = r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7;   // never taken
}

__global__ __launch_bounds__(PROBE_THREADS) void probe_read_b64(int iters, uint32_t* out)
{
  const uint32_t a = threadIdx.x * 8u;   // < 2 KB; offsets up to 6 KB
  u32x2 r0, r1, r2, r3, r4, r5, r6, r7;
  for (int i = 0; i < iters; ++i) {
    asm volatile(
        "ds_read_b64 %0, %8\n"
        "ds_read_b64 %1, %8 offset:2048\n"
        "ds_read_b64 %2, %8 offset:4096\n"
        "ds_read_b64 %3, %8 offset:6144\n"
        "ds_read_b64 %4, %8\n"
        "ds_read_b64 %5, %8 offset:2048\n"
        "ds_read_b64 %6, %8 offset:4096\n"
        "ds_read_b64 %7, %8 offset:6144\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(a)
        : "memory");
  }
  if (iters < 0) out[threadIdx.x] = (r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7).x;
}

__global__ __launch_bounds__(PROBE_THREADS) void probe_read_b128(int iters, uint32_t* out)
{
  const uint32_t a = threadIdx.x * 16u;   // < 4 KB; offsets up to 4 KB
  u32x4 r0, r1, r2, r3, r4, r5, r6, r7;
  for (int i = 0; i < iters; ++i) {
    asm volatile(
        "ds_read_b128 %0, %8\n"
        "ds_read_b128 %1, %8 offset:4096\n"
        "ds_read_b128 %2, %8\n"
        "ds_read_b128 %3, %8 offset:4096\n"
        "ds_read_b128 %4, %8\n"
        "ds_read_b128 %5, %8 offset:4096\n"
        "ds_read_b128 %6, %8\n"
        "ds_read_b128 %7, %8 offset:4096\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)
        : "v"(a)
        : "memory");
  }
  if (iters < 0) out[threadIdx.x] = (r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7).x;
}

__global__ __launch_bounds__(PROBE_THREADS) void probe_write_b32(int iters, uint32_t* out)
{
  const uint32_t a = threadIdx.x * 4u;
  uint32_t v = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
    asm volatile(
        "ds_write_b32 %0, %1\n"
        "ds_write_b32 %0, %1 offset:1024\n"
        "ds_write_b32 %0, %1 offset:2048\n"
        "ds_write_b32 %0, %1 offset:3072\n"
        "ds_write_b32 %0, %1 offset:4096\n"
        "ds_write_b32 %0, %1 offset:5120\n"
        "ds_write_b32 %0, %1 offset:6144\n"
        "ds_write_b32 %0, %1 offset:7168\n"
        "s_waitcnt lgkmcnt(0)\n"
        :
        : "v"(a), "v"(v)
        : "memory");
  }
  if (iters < 0) out[threadIdx.x] = v;
}

__global__ __launch_bounds__(PROBE_THREADS) void probe_write_b64(int iters, uint32_t* out)
{
  const uint32_t a = threadIdx.x * 8u;
  u32x2 v = {threadIdx.x, threadIdx.x + 1u};
  for (int i = 0; i < iters; ++i) {
    asm volatile(
        "ds_write_b64 %0, %1\n"
        "ds_write_b64 %0, %1 offset:2048\n"
        "ds_write_b64 %0, %1 offset:4096\n"
        "ds_write_b64 %0, %1 offset:6144\n"
        "ds_write_b64 %0, %1\n"
        "ds_write_b64 %0, %1 offset:2048\n"
        "ds_write_b64 %0, %1 offset:4096\n"
        "ds_write_b64 %0, %1 offset:6144\n"
        "s_waitcnt lgkmcnt(0)\n"
        :
        : "v"(a), "v"(v)
        : "memory");
  }
  if (iters < 0) out[threadIdx.x] = v.x;
}

__global__ __launch_bounds__(PROBE_THREADS) void probe_write_b128(int iters, uint32_t* out)
{
  const uint32_t a = threadIdx.x * 16u;
  u32x4 v = {threadIdx.x, threadIdx.x + 1u, threadIdx.x + 2u, threadIdx.x + 3u};
  for (int i = 0; i < iters; ++i) {
    asm volatile(
        "ds_write_b128 %0, %1\n"
        "ds_write_b128 %0, %1 offset:4096\n"
        "ds_write_b128 %0, %1\n"
        "ds_write_b128 %0, %1 offset:4096\n"
        "ds_write_b128 %0, %1\n"
        "ds_write_b128 %0, %1 offset:4096\n"
        "ds_write_b128 %0, %1\n"
        "ds_write_b128 %0, %1 offset:4096\n"
        "s_waitcnt lgkmcnt(0)\n"
        :
        : "v"(a), "v"(v)
        : "memory");
  }
  if (iters < 0) out[threadIdx.x] = v.x;
}

typedef void (*probe_fn)(int, uint32_t*);

probe_fn pick(int kind, int width)
{
  if (kind == LDS_PROBE_READ) {
    if (width == 4) return probe_read_b32;
    if (width == 8) return probe_read_b64;
    if (width == 16) return probe_read_b128;
  } else if (kind == LDS_PROBE_WRITE) {
    if (width == 4) return probe_write_b32;
    if (width == 8) return probe_write_b64;
    if (width == 16) return probe_write_b128;
  }
  return nullptr;
}

}  // namespace

extern "C" {

int lds_probe_run(int32_t kind, int32_t width, int32_t blocks_per_cu, int32_t iters, void* stream,
                  double* bytes_per_s, float* ms_out)
{
  probe_fn fn = pick(kind, width);
  if (!fn || blocks_per_cu < 1 || blocks_per_cu > 64 || iters < 1 || !bytes_per_s) return -1;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return -4;
  const int grid = prop.multiProcessorCount * blocks_per_cu;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -4;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -4;
  }
  int rc = 0;
  // one untimed launch, then the timed one
  for (int rep = 0; rep < 2 && !rc; ++rep) {
    if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = -4;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(PROBE_THREADS), PROBE_LDS_BYTES, st, iters, (uint32_t*)nullptr);
    if (!rc && hipGetLastError() != hipSuccess) rc = -4;
    if (rep == 1 && !rc && hipEventRecord(e1, st) != hipSuccess) rc = -4;
  }
  float ms = 0.f;
  if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) rc = -4;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const double bytes = (double)grid * PROBE_THREADS * (double)iters * PROBE_GROUP * width;
  *bytes_per_s = bytes / (ms * 1e-3);
  if (ms_out) *ms_out = ms;
  return 0;
}

}  // extern "C"
