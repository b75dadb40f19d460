// kernels.hip -- time-record kernels, the rate-kernel launcher and the
// stage-launch dispatcher.  The stage kernels themselves (stage_kernels.h) are
// instantiated by kernels_inst.hip, which the build compiles once per
// (dimension, precision, stage) so that the instantiations build in parallel.
#include "stage_kernels.h"

namespace hyd {

// Stage launchers of the instantiation units, one per (dimension, mixed, stage).
#define HYD_DECL(D, M, S)                                                                                     \
  hipError_t launch_stage_inst_##D##_##M##_##S(int kmask, int speeds, int recon, int eos, int occ, int grid,      \
                                               hipStream_t s, const StageArgs &a);
HYD_DECL(2, 0, 1)
HYD_DECL(2, 0, 2)
HYD_DECL(2, 1, 1)
HYD_DECL(2, 1, 2)
HYD_DECL(3, 0, 1)
HYD_DECL(3, 0, 2)
HYD_DECL(3, 1, 1)
HYD_DECL(3, 1, 2)
#undef HYD_DECL

__global__ void k_reset(DevTime *t) {
  t->lam_bits = 0ull;
  t->status = 0;
  t->bad_block = INT_MAX;
}

// After a step (init = 0): t += dt; dt = cfl / rate of the new state.
// Before the first step (init = 1): t = 0; dt = cfl / rate.
// Once a non-physical state was seen, dt is NaN and stays NaN (the status is
// not cleared within a run): the stage launches of later steps then do
// nothing and t keeps the time of the failing step.
__global__ void k_finalize(DevTime *t, double cfl, int init) {
  const double lam = __longlong_as_double((long long)t->lam_bits);
  if (init) {
    t->t = 0.0;
  } else {
    if (!(__builtin_fabs(t->dt) <= __DBL_MAX__)) {
      t->lam_bits = 0ull;
      return;
    }
    t->t += t->dt;
  }
  t->dt = (t->status == 0 && lam > 0.0) ? cfl / lam : __builtin_nan("");
  t->lam_bits = 0ull;
}

// ------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------
hipError_t launch_stage(int ndim, bool mixed, int stage, int kmask, int speeds, int recon, int eos, int grid,
                        hipStream_t s, const StageArgs &a, int occ) {
  if (grid <= 0) return hipSuccess;
  if (eos == EOS_GAS_RADIATION && (mixed || speeds != SPEEDS_DAVIS || recon != RECON_PRIMITIVE))
    return hipErrorInvalidValue;  // FP64, Davis bounds, primitive PLM only (checked by the caller)
  if (occ != 0 && (occ < 2 || occ > 4)) return hipErrorInvalidValue;
  const int k = kmask, w = speeds, r = recon, e = eos, o = occ;
  if (ndim == 2) {
    if (mixed)
      return stage == 1 ? launch_stage_inst_2_1_1(k, w, r, e, o, grid, s, a) : launch_stage_inst_2_1_2(k, w, r, e, o, grid, s, a);
    return stage == 1 ? launch_stage_inst_2_0_1(k, w, r, e, o, grid, s, a) : launch_stage_inst_2_0_2(k, w, r, e, o, grid, s, a);
  }
  if (mixed)
    return stage == 1 ? launch_stage_inst_3_1_1(k, w, r, e, o, grid, s, a) : launch_stage_inst_3_1_2(k, w, r, e, o, grid, s, a);
  return stage == 1 ? launch_stage_inst_3_0_1(k, w, r, e, o, grid, s, a) : launch_stage_inst_3_0_2(k, w, r, e, o, grid, s, a);
}

template <int EOS, bool MIXED>
static void launch_lambda_e(int ndim, bool t16, int grid, hipStream_t s, const StageArgs &a) {
  if (ndim == 2) {
    if (t16)
      hipLaunchKernelGGL((k_lambda<2, 3, EOS, MIXED>), dim3(grid), dim3(WG), 0, s, a);
    else
      hipLaunchKernelGGL((k_lambda<2, 2, EOS, MIXED>), dim3(grid), dim3(WG), 0, s, a);
  } else {
    if (t16)
      hipLaunchKernelGGL((k_lambda<3, 3, EOS, MIXED>), dim3(grid), dim3(WG), 0, s, a);
    else
      hipLaunchKernelGGL((k_lambda<3, 2, EOS, MIXED>), dim3(grid), dim3(WG), 0, s, a);
  }
}

hipError_t launch_lambda(int ndim, bool mixed, int kmask, int eos, int grid, hipStream_t s, const StageArgs &a) {
  if (grid <= 0) return hipSuccess;
  const bool t16 = kmask & 1;
  if (eos == EOS_GAS_RADIATION) {
    if (mixed) return hipErrorInvalidValue;  // FP64 only
    launch_lambda_e<EOS_GAS_RADIATION, false>(ndim, t16, grid, s, a);
  } else if (mixed) {
    launch_lambda_e<EOS_IDEAL, true>(ndim, t16, grid, s, a);
  } else {
    launch_lambda_e<EOS_IDEAL, false>(ndim, t16, grid, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fused(bool mixed, int grid, hipStream_t s, const FusedArgs &a) {
  if (grid <= 0) return hipSuccess;
  if (mixed)
    hipLaunchKernelGGL((k_fused_cube8<true>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_fused_cube8<false>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

// The host share's CFL rate and non-physical flag, merged into the
// accumulator (before the dt update of the step).
__global__ void k_fold(DevTime *t, double lam, int bad, int bad_block) {
  atomicMax(&t->lam_bits, (unsigned long long)__double_as_longlong(lam));
  if (bad) {
    atomicOr(&t->status, 1);
    atomicMin(&t->bad_block, bad_block);
  }
}

hipError_t launch_fold(DevTime *t, double lam, int bad, int bad_block, hipStream_t s) {
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(1), 0, s, t, lam, bad, bad_block);
  return hipGetLastError();
}

hipError_t launch_reset(DevTime *t, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_finalize(DevTime *t, double cfl, int init, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1), 0, s, t, cfl, init);
  return hipGetLastError();
}

}  // namespace hyd
