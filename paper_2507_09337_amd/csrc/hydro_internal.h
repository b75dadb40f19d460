// Internal types shared by the HIP kernels (kernels.hip) and the host library
// (api.hip).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyd {

constexpr int NVAR = 5;
constexpr int WG = 256;  // threads per workgroup of every stage kernel

// Device copy of one block, with the guard sources of its six faces resolved.
// Face f (-x,+x,-y,+y,-z,+z) copies its two guard layers from block
// data at element offset foff[f]: that block's extent along the face axis is
// fnax[f], its cell count fnc[f].  fmode[f] = 0: wrap (the far layers of the
// source, which is a linked neighbour or the block itself); 1: outflow (the
// edge layer of the block itself, repeated).
struct DevBlock {
  int64_t off;
  int32_t n[3];
  int32_t ncell;
  double dx[3];
  int64_t foff[6];
  int32_t fnax[6];
  int32_t fnc[6];
  int32_t fmode[6];
  int32_t pad[2];
};

// One work item of a stage launch: x-y tiles, each marched over z planes
// [z0, z1).  kind 0: a run of up to four 16x16 tiles (block[s], x0[s],
// y0[s]) taken one after the other by the whole workgroup, block[s] < 0
// ending the run; kind 1: up to four 8x8 tiles, one per 64-thread wave, from
// any blocks (block[s] < 0 = empty).
struct WorkItem {
  int32_t block[4];
  int16_t x0[4];
  int16_t y0[4];
  int16_t z0, z1;
  int32_t kind;
};

enum { KIND_T16 = 0, KIND_T8 = 1 };

// Device-resident step bookkeeping of a packet or batch.
struct DevTime {
  double dt;                    // time step used by the next stage launches (graph path)
  double t;                     // simulated time advanced by the graph path
  unsigned long long lam_bits;  // max CFL rate as the bits of a non-negative double
  int32_t status;               // nonzero: a non-physical state was seen
  int32_t bad_block;            // smallest block id with a non-physical state
};

struct StageArgs {
  const DevBlock *blocks;
  const WorkItem *items;
  int32_t nitems;
  int32_t reset_time;  // 1: workgroup 0 clears lam/status of `acc` first (plain path)
  int32_t xcd_remap;   // 1: give each XCD a contiguous span of the work list
  const double *src;   // state the fluxes are computed from (Un or U1)
  const double *un;    // Un (stage 2 only)
  double *dst;         // U1 (stage 1) or Un+1 (stage 2, may alias un)
  double dt;           // used when dt_dev is null
  const DevTime *dt_dev;
  DevTime *acc;        // CFL rate and status accumulator
  double gamma;
};

// Arguments of the fused step of self-periodic 8^3 blocks (one workgroup per
// listed block; Un+1 overwrites Un in place).
struct FusedArgs {
  const DevBlock *blocks;
  const int32_t *ids;  // the blocks the fused kernel takes
  int32_t nblocks;
  int32_t rate_only;   // 1: only reduce the CFL rate of the current state into acc
  int32_t xcd_remap;
  double *state;
  double dt;           // used when dt_dev is null
  const DevTime *dt_dev;
  DevTime *acc;
  double gamma;
};

// kmask: bit 0 = the launch contains 16x16 items, bit 1 = 8x8 items.
// speeds: 0 = Davis, 1 = Einfeldt, 2 = pressure-based (PVRS) wave-speed bounds in HLLC.
// recon: 0 = PLM on primitives, 1 = on conserved variables, 2 = on characteristic variables.
// eos: 0 = gamma law, 1 = gas + radiation (FP64 with Davis bounds and primitive PLM only).
// occ: 0 = the kernels' own register budget; 2, 3 or 4 = at least that many
// waves per SIMD (default method only; the variants keep their own).
hipError_t launch_stage(int ndim, bool mixed, int stage, int kmask, int speeds, int recon, int eos, int grid,
                        hipStream_t s, const StageArgs &a, int occ = 0);
// mixed: the rate as the mixed path's stage 2 reduces it (refined hardware
// reciprocal and reciprocal square root); else in oracle order.
hipError_t launch_lambda(int ndim, bool mixed, int kmask, int eos, int grid, hipStream_t s, const StageArgs &a);
hipError_t launch_fused(bool mixed, int grid, hipStream_t s, const FusedArgs &a);
hipError_t launch_fold(DevTime *t, double lam, int bad, int bad_block, hipStream_t s);
hipError_t launch_reset(DevTime *t, hipStream_t s);
hipError_t launch_finalize(DevTime *t, double cfl, int init, hipStream_t s);

}  // namespace hyd
