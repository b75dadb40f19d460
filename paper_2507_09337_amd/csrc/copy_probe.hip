// copy_probe.hip -- measurement helper, not part of the hydro path.
//
// Plain device-to-device copies of n doubles, used (1) to measure the HBM
// bandwidth a streaming kernel reaches on this GPU (buffers far larger than
// the 256 MB last-level cache) and (2) as the "copy kernel of known size"
// whose FETCH_SIZE / WRITE_SIZE counters calibrate the counters read on the
// stage kernels.  Two forms: one 16-byte element per thread and iteration
// (k_copy), and four independent 16-byte elements per thread in flight before
// any store, with nontemporal accesses (k_copy4).
#include <hip/hip_runtime.h>
#include <stdint.h>

__global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

// n2 must be a multiple of 1024 (4 elements x 256 threads per workgroup step)
__global__ __launch_bounds__(256) void k_copy4(const dvec2 *__restrict__ src, dvec2 *__restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * 1024;
  for (int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x; base < n2; base += stride) {
    dvec2 a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = __builtin_nontemporal_load(src + base + 256 * k);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(a[k], dst + base + 256 * k);
  }
}

extern "C" {

// Copies n doubles (n a multiple of 2048 for form 1; both pointers 16-byte
// aligned device pointers) reps times on `stream` with kernel form `form`
// (0: k_copy, 1: k_copy4); returns the mean time per copy in ms through
// ms_out (host pointer).  Returns 0 on success, 1 on bad arguments, 2 on a
// HIP error.
int copy_probe(const double *src, double *dst, int64_t n, void *stream, int reps, int form, double *ms_out) {
  if (!src || !dst || !ms_out || n <= 0 || (n & 1) || reps < 1 || (form != 0 && form != 1)) return 1;
  if (form == 1 && (n % 2048)) return 1;
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return 1;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2;
  const int64_t n2 = n / 2;
  const int64_t per = form ? 1024 : 256;
  const int64_t want = (n2 + per - 1) / per;
  const int grid = (int)(want < (int64_t)ncu * 16 ? want : (int64_t)ncu * 16);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 2;
  auto launch = [&]() {
    if (form)
      hipLaunchKernelGGL(k_copy4, dim3(grid), dim3(256), 0, s, (const dvec2 *)src, (dvec2 *)dst, n2);
    else
      hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, (const double2 *)src, (double2 *)dst, n2);
  };
  launch();  // warm-up
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, s);
  int rc = 0;
  if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) rc = 2;
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = ms / reps;
  return rc;
}
}
