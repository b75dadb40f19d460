// Host-core kernel of the CPU/GPU split of host-resident packets
// (host_step.hip).  Not part of the ABI.
#pragma once
#include <climits>
#include <vector>

#include "hydro.h"

namespace hyd {

// One RK stage (or the CFL rate) of the blocks `ids` on the host, FP64,
// Davis bounds, primitive PLM, gamma law.  Per block b (global id into desc):
// src[b] is the stage source (variable 0 of the block; layout of the arena),
// un[b] the state Un (stage 2), dst[b] the result (U1 after stage 1, Un+1
// after stage 2; never a block some other block reads as its source in the
// same stage).  Guard rules as on the GPU: linked faces read src[nbr].
struct HostStage {
  const hydro_block_desc *desc = nullptr;
  int ndim = 3;
  int stage = 1;
  std::vector<int32_t> ids;
  const double *const *src = nullptr;
  const double *const *un = nullptr;
  double *const *dst = nullptr;
  double dt = 0.0;
  double gamma = 1.4;
};

// Largest CFL rate of the new state (stage 2) or of the source (rate only),
// and whether a non-physical state was seen (stage 2: the first-stage state
// or the new state; rate: the source), with the smallest block id concerned.
struct HostRate {
  double lam = 0.0;
  int bad = 0;
  int bad_block = INT_MAX;
};

HostRate host_run(const HostStage &h, int nthreads, bool rate_only);

}  // namespace hyd
