// copy_probe.hip -- measurement helper, not part of the hydro path.
//
// A plain device-to-device copy of n doubles with 16-byte vector loads and
// stores, used (1) to measure the HBM bandwidth a streaming kernel reaches on
// this GPU (buffers far larger than the 256 MB last-level cache), and (2) as
// the "copy kernel of known size" whose FETCH_SIZE / WRITE_SIZE counters
// calibrate the counters read on the stage kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

__global__ __launch_bounds__(256) void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

extern "C" {

// Copies n doubles (n even, both pointers 16-byte aligned device pointers)
// reps times on `stream`; returns the mean time per copy in ms through
// ms_out (host pointer).  Returns 0 on success, 1 on bad arguments, 2 on a
// HIP error.
int copy_probe(const double *src, double *dst, int64_t n, void *stream, int reps, double *ms_out) {
  if (!src || !dst || !ms_out || n <= 0 || (n & 1) || reps < 1) return 1;
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return 1;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2;
  const int64_t n2 = n / 2;
  int64_t want = (n2 + 255) / 256;
  const int grid = (int)(want < (int64_t)ncu * 16 ? want : (int64_t)ncu * 16);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 2;
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, (const double2 *)src, (double2 *)dst, n2);  // warm-up
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, (const double2 *)src, (double2 *)dst, n2);
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
