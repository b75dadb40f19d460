// kernels_inst.hip -- instantiation unit of the stage kernels for one
// (dimension, precision, stage), chosen by HYD_DIM, HYD_MIXED and HYD_STAGE
// on the compiler command line (the build compiles this file once for each
// of the eight combinations).
#include "stage_kernels.h"

#if !defined(HYD_DIM) || !defined(HYD_MIXED) || !defined(HYD_STAGE)
#error "kernels_inst.hip needs -DHYD_DIM=2|3 -DHYD_MIXED=0|1 -DHYD_STAGE=1|2"
#endif

#define HYD_CAT2(D, M, S) launch_stage_inst_##D##_##M##_##S
#define HYD_CAT(D, M, S) HYD_CAT2(D, M, S)

namespace hyd {

hipError_t HYD_CAT(HYD_DIM, HYD_MIXED, HYD_STAGE)(int kmask, int speeds, int recon, int eos, int occ, int grid,
                                                   hipStream_t s, const StageArgs &a) {
  constexpr int D = HYD_DIM, S = HYD_STAGE;
  constexpr bool M = HYD_MIXED != 0;
  if (eos == EOS_GAS_RADIATION) {
    if constexpr (M) {
      return hipErrorInvalidValue;  // the gas + radiation EOS runs on the FP64 tile only
    } else {
      return launch_ks<D, false, S, SPEEDS_DAVIS, RECON_PRIMITIVE, EOS_GAS_RADIATION>(kmask, grid, s, a);
    }
  }
  if (occ > 0 && speeds == SPEEDS_DAVIS && recon == RECON_PRIMITIVE) return launch_occ<D, M, S>(kmask, occ, grid, s, a);
  return launch_k<D, M, S>(kmask, speeds, recon, grid, s, a);
}

}  // namespace hyd
