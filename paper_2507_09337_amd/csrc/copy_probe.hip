// copy_probe.hip -- measurement helper, not part of the hydro path.
//
// Plain streaming kernels over buffers far larger than the 256 MB last-level
// cache, used (1) to find the HBM bandwidth a streaming kernel reaches on
// this GPU -- the practical ceiling the stage kernels are compared with --
// and (2) as the "copy kernel of known size" whose FETCH_SIZE / WRITE_SIZE
// counters calibrate the counters read on the stage kernels.
//
// Kernel forms, each with E independent 16-byte elements per thread in
// flight (all loads issued before the first store) and a grid of G
// workgroups of 256 threads looping over the buffer:
//   copy  (mode 0): dst = src, plain accesses;
//   copy  (mode 1): dst = src, nontemporal loads and stores;
//   read  (mode 2): sum of src per thread, one store per thread at the end;
//   write (mode 3): dst = a constant, nontemporal stores.
// The sweep varies E in {1, 2, 4, 8}, G in {2..32} x CUs and the buffer size.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int E, bool NT>
__global__ __launch_bounds__(256) void k_copy_e(const dvec2 *__restrict__ src, dvec2 *__restrict__ dst, int64_t n2) {
  const int64_t step = (int64_t)256 * E;
  const int64_t stride = (int64_t)gridDim.x * step;
  for (int64_t base = (int64_t)blockIdx.x * step + threadIdx.x; base < n2; base += stride) {
    dvec2 a[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int64_t i = base + 256 * k;
      if (i < n2) a[k] = NT ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int64_t i = base + 256 * k;
      if (i < n2) {
        if (NT)
          __builtin_nontemporal_store(a[k], dst + i);
        else
          dst[i] = a[k];
      }
    }
  }
}

// out holds one dvec2 per thread of the grid.
template <int E>
__global__ __launch_bounds__(256) void k_read_e(const dvec2 *__restrict__ src, dvec2 *__restrict__ out, int64_t n2) {
  const int64_t step = (int64_t)256 * E;
  const int64_t stride = (int64_t)gridDim.x * step;
  dvec2 acc = {0.0, 0.0};
  for (int64_t base = (int64_t)blockIdx.x * step + threadIdx.x; base < n2; base += stride) {
    dvec2 a[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int64_t i = base + 256 * k;
      a[k] = (i < n2) ? __builtin_nontemporal_load(src + i) : dvec2{0.0, 0.0};
    }
#pragma unroll
    for (int k = 0; k < E; ++k) acc += a[k];
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

template <int E>
__global__ __launch_bounds__(256) void k_write_e(dvec2 *__restrict__ dst, int64_t n2, double v) {
  const int64_t step = (int64_t)256 * E;
  const int64_t stride = (int64_t)gridDim.x * step;
  const dvec2 x = {v, v};
  for (int64_t base = (int64_t)blockIdx.x * step + threadIdx.x; base < n2; base += stride) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int64_t i = base + 256 * k;
      if (i < n2) __builtin_nontemporal_store(x, dst + i);
    }
  }
}

template <int E>
static void launch_e(int mode, int grid, hipStream_t s, const double *src, double *dst, int64_t n2) {
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((k_copy_e<E, false>), dim3(grid), dim3(256), 0, s, (const dvec2 *)src, (dvec2 *)dst, n2);
      break;
    case 1:
      hipLaunchKernelGGL((k_copy_e<E, true>), dim3(grid), dim3(256), 0, s, (const dvec2 *)src, (dvec2 *)dst, n2);
      break;
    case 2:
      hipLaunchKernelGGL((k_read_e<E>), dim3(grid), dim3(256), 0, s, (const dvec2 *)src, (dvec2 *)dst, n2);
      break;
    default:
      hipLaunchKernelGGL((k_write_e<E>), dim3(grid), dim3(256), 0, s, (dvec2 *)dst, n2, 1.0);
      break;
  }
}

extern "C" {

// One form of the sweep: mode 0..3 as above, `elems` in {1, 2, 4, 8} 16-byte
// elements per thread in flight, `wg_per_cu` workgroups per CU (grid =
// wg_per_cu x CUs, capped at the work), over n doubles (n even; both pointers
// 16-byte aligned device pointers; for mode 2, dst must hold 2 doubles per
// thread of the grid, i.e. 512 x grid doubles).  Runs one warm-up and `reps`
// timed launches on `stream`; *ms_out (host) receives the mean time per
// launch in ms.  Returns 0 on success, 1 on bad arguments, 2 on a HIP error.
int stream_probe(const double *src, double *dst, int64_t n, void *stream, int reps, int mode, int elems,
                 int wg_per_cu, double *ms_out) {
  if (!dst || !ms_out || n <= 0 || (n & 1) || reps < 1 || mode < 0 || mode > 3 || wg_per_cu < 1) return 1;
  if (mode != 3 && !src) return 1;
  if (elems != 1 && elems != 2 && elems != 4 && elems != 8) return 1;
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return 1;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2;
  const int64_t n2 = n / 2;
  const int64_t per = (int64_t)256 * elems;
  const int64_t want = (n2 + per - 1) / per;
  const int64_t cap = (int64_t)ncu * wg_per_cu;
  const int grid = (int)(want < cap ? want : cap);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 2;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 2;
  }
  auto launch = [&]() {
    switch (elems) {
      case 1: launch_e<1>(mode, grid, s, src, dst, n2); break;
      case 2: launch_e<2>(mode, grid, s, src, dst, n2); break;
      case 4: launch_e<4>(mode, grid, s, src, dst, n2); break;
      default: launch_e<8>(mode, grid, s, src, dst, n2); break;
    }
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

// The calibration copy of the counter summaries: form 0 = plain copy, one
// element per thread, 16 workgroups per CU; form 1 = nontemporal copy, four
// elements per thread in flight, 16 workgroups per CU.
int copy_probe(const double *src, double *dst, int64_t n, void *stream, int reps, int form, double *ms_out) {
  if (form != 0 && form != 1) return 1;
  return stream_probe(src, dst, n, stream, reps, form, form ? 4 : 1, 16, ms_out);
}
}
