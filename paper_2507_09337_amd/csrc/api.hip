// api.hip -- host side of the C ABI declared in include/hydro.h.
//
// Owns descriptor validation (entirely on the host, before any HIP call),
// the device block table, the work lists of packets and batches, the
// stage-synchronous plain path, the HIP-graph batched path and the autotuner.
// Kernels live in kernels.hip.
#include <algorithm>
#include <array>
#include <chrono>
#include <cfloat>
#include <climits>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "host_step.h"
#include "hydro.h"
#include "hydro_internal.h"

using hyd::DevBlock;
using hyd::DevTime;
using hyd::StageArgs;
using hyd::WorkItem;

namespace {

// Message of the last failing call on this thread: a fixed buffer, so that
// reporting an error never allocates.
thread_local char g_err[512];

hydro_status failf(hydro_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
hydro_status failf(hydro_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

hydro_status fail(hydro_status s, const std::string &msg) { return failf(s, "%s", msg.c_str()); }

#define HIP_TRY(call)                                                                                 \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return fail(HYDRO_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

struct TileCfg {
  int tile = -1;   // -1: default (16x16 when the extents allow it); 0: 16x16; 1: 8x8;
                   // 2..4: 16x16 in runs of that many blocks along +z;
                   // 5: fused step (self-periodic 8^3 blocks, both stages in one launch)
  int zchunk = 0;  // 0: whole block
};

constexpr int TILE_FUSED = 5;

// A block the fused step can take: 3D, 8^3 interior cells, every face
// periodic on the block itself.
bool fusable(const hydro_block_desc &d, int ndim) {
  if (ndim != 3 || d.n[0] != 8 || d.n[1] != 8 || d.n[2] != 8) return false;
  for (int f = 0; f < 6; ++f)
    if (d.face_kind[f] != HYDRO_PERIODIC_SELF) return false;
  return true;
}

// Class of a block for tuning: its edge when the block is a square (2D) or a
// cube (3D), else 0.
int block_class(const hydro_block_desc &d, int ndim) {
  if (d.n[0] != d.n[1]) return 0;
  if (ndim == 3 && d.n[2] != d.n[0]) return 0;
  return d.n[0];
}

}  // namespace

struct hydro_mesh {
  int device = 0;
  hipStream_t stream = nullptr;
  int ndim = 3;
  int nblocks = 0;
  double *arena = nullptr;
  int64_t arena_len = 0;
  double *u1 = nullptr;  // first-stage state, same layout as the arena
  DevBlock *d_blocks = nullptr;
  std::vector<hydro_block_desc> desc;
  int children = 0;  // live packets and batches
  int num_cu = 0;
};

struct WorkList {
  WorkItem *d_items = nullptr;
  int nitems = 0;
  int kmask = 0;
};

struct hydro_packet {
  hydro_mesh *m = nullptr;
  std::vector<int32_t> ids;
  int prec = HYDRO_FP64;
  WorkList wl;
  DevTime *d_time = nullptr;
  bool closed = false;
  bool lam_valid = false;  // the last call was an advance: d_time holds the rate of the new state
  double lam_gamma = 0.0;
  int batches = 0;
};

struct hydro_batch {
  hydro_mesh *m = nullptr;
  std::vector<hydro_packet *> packets;
  std::vector<int32_t> ids;  // all blocks, packet order
  int prec = HYDRO_FP64;
  std::map<int, TileCfg> cfg;
  int grid = 0;
  int remap = 1;
  int occ = 0;  // waves per SIMD asked of the stage kernels (0 = their own budget)
  WorkList wl;
  int32_t *d_fused = nullptr;  // blocks taken by the fused step (classes tiled TILE_FUSED)
  int nfused = 0;
  DevTime *d_time = nullptr;
  hipStream_t cap_stream = nullptr;
  hipStream_t side_stream = nullptr;  // the fused launch's branch of a captured step
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double g_cfl = 0.0, g_gamma = 0.0;
};

namespace {

// ---------------------------------------------------------------- validation
// Checks of one block descriptor (everything but overlap with other blocks):
// nullptr if it is valid, else a message; *face receives the face concerned
// (-1 if none).
const char *block_error(const hydro_block_desc *blocks, int32_t nb, int32_t ndim, int64_t arena_len, int b,
                        int *face) {
  const hydro_block_desc &d = blocks[b];
  *face = -1;
  if (d.reserved != 0) return "reserved field must be 0";
  if (d.n[0] < 8 || d.n[1] < 8 || d.n[0] % 8 || d.n[1] % 8) return "n[0] and n[1] must be positive multiples of 8";
  if (d.n[0] > 16384 || d.n[1] > 16384) return "n[0], n[1] must be <= 16384";
  if (ndim == 2 && d.n[2] != 1) return "n[2] must be 1 in 2D";
  if (ndim == 3 && (d.n[2] < 2 || d.n[2] > 16384)) return "n[2] must be in [2, 16384] in 3D";
  const int64_t nc = (int64_t)d.n[0] * d.n[1] * d.n[2];
  if (nc >= ((int64_t)1 << 31)) return "too many cells";
  for (int a = 0; a < ndim; ++a)
    if (!finite_pos(d.dx[a])) return "dx must be finite and > 0";
  if (d.offset < 0 || d.offset > arena_len - 5 * nc) return "range outside the arena";
  for (int f = 0; f < 2 * ndim; ++f) {
    *face = f;
    const int k = d.face_kind[f];
    if (k != HYDRO_NBR && k != HYDRO_OUTFLOW && k != HYDRO_PERIODIC_SELF) return "bad face kind";
    if (k != HYDRO_NBR) continue;
    const int s = d.nbr[f];
    if (s < 0 || s >= nb) return "neighbour id out of range";
    const int axis = f / 2;
    for (int a = 0; a < 3; ++a)
      if (a != axis && blocks[s].n[a] != d.n[a]) return "neighbour has other tangential extents";
    if (blocks[s].n[axis] < 2) return "neighbour too thin for two guard layers";
  }
  *face = -1;
  return nullptr;
}

// Descriptor checks of a mesh; `ranges` (nb entries of scratch, owned by the
// caller) is sorted to find overlapping blocks.
hydro_status validate_blocks(const hydro_block_desc *blocks, int32_t nb, int32_t ndim, const double *arena,
                             int64_t arena_len, std::pair<int64_t, int64_t> *ranges) {
  if (nb <= 0 || !blocks) return failf(HYDRO_EINVAL, "mesh: nblocks must be > 0 and blocks non-null");
  if (ndim != 2 && ndim != 3) return failf(HYDRO_EINVAL, "mesh: ndim must be 2 or 3");
  if (!arena || arena_len <= 0) return failf(HYDRO_EINVAL, "mesh: arena must be non-null with arena_len > 0");
  for (int b = 0; b < nb; ++b) {
    int face = -1;
    if (const char *why = block_error(blocks, nb, ndim, arena_len, b, &face)) {
      if (face >= 0) return failf(HYDRO_EINVAL, "mesh: block %d: %s on face %d", b, why, face);
      return failf(HYDRO_EINVAL, "mesh: block %d: %s", b, why);
    }
    const hydro_block_desc &d = blocks[b];
    ranges[b] = {d.offset, d.offset + 5 * (int64_t)d.n[0] * d.n[1] * d.n[2]};
  }
  std::sort(ranges, ranges + nb);
  for (int i = 1; i < nb; ++i)
    if (ranges[i].first < ranges[i - 1].second) return failf(HYDRO_EINVAL, "mesh: block ranges overlap in the arena");
  return HYDRO_OK;
}

hydro_status validate_mesh(const hydro_block_desc *blocks, int32_t nb, int32_t ndim, const double *arena,
                           int64_t arena_len) {
  std::vector<std::pair<int64_t, int64_t>> ranges(nb > 0 ? nb : 0);
  return validate_blocks(blocks, nb, ndim, arena, arena_len, ranges.data());
}

DevBlock make_devblock(const hydro_block_desc *all, int b, int ndim) {
  const hydro_block_desc &d = all[b];
  DevBlock B;
  std::memset(&B, 0, sizeof(B));
  B.off = d.offset;
  for (int a = 0; a < 3; ++a) {
    B.n[a] = d.n[a];
    B.dx[a] = (a < ndim) ? d.dx[a] : 1.0;
  }
  B.ncell = d.n[0] * d.n[1] * d.n[2];
  for (int f = 0; f < 6; ++f) {
    const int axis = f / 2;
    int kind = (f < 2 * ndim) ? d.face_kind[f] : HYDRO_OUTFLOW;
    const int src = (kind == HYDRO_NBR) ? d.nbr[f] : b;
    const hydro_block_desc &s = all[src];
    B.foff[f] = s.offset;
    B.fnax[f] = s.n[axis];
    B.fnc[f] = s.n[0] * s.n[1] * s.n[2];
    B.fmode[f] = (kind == HYDRO_OUTFLOW) ? 1 : 0;
  }
  return B;
}

// ---------------------------------------------------------------- work lists
// Default z-run length of a class of whole 16x16-tiled 3D blocks with
// `tiles` tiles: two when the halved work list still gives two or more rounds
// of resident workgroups (three per CU), else one.  Measured: runs of two win
// from 2.7 rounds up (4096 and 32768 tiles of 16^3 blocks); below two rounds
// the idle share of the last round outweighs the saved z halo.
int default_run(const hydro_mesh *m, int64_t tiles) {
  return (m->ndim == 3 && m->num_cu > 0 && tiles / 2 >= 2 * 3 * (int64_t)m->num_cu) ? 2 : 1;
}

// Work of an item in cell-planes: the planes it marches times the cells of
// its tiles.
int64_t item_cost(const hydro_mesh *m, const WorkItem &it) {
  int64_t c = 0;
  for (int s = 0; s < 4; ++s) {
    if (it.block[s] < 0) continue;
    const int planes = it.kind == hyd::KIND_T16 && s > 0 ? m->desc[it.block[s]].n[2] : it.z1 - it.z0;
    c += (int64_t)planes * (it.kind == hyd::KIND_T16 ? 256 : 64);
  }
  return c;
}

// Heaviest items first (a stable sort: items of equal work keep the block
// order that puts neighbouring blocks next to each other).  On uneven blocks
// the big items then start in the first rounds and the small ones fill the
// last, instead of a few big items running alone at the end of a launch.
void order_items(const hydro_mesh *m, std::vector<WorkItem> &items) {
  std::vector<int64_t> cost(items.size());
  for (size_t i = 0; i < items.size(); ++i) cost[i] = item_cost(m, items[i]);
  std::vector<size_t> idx(items.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<WorkItem> out(items.size());
  for (size_t i = 0; i < idx.size(); ++i) out[i] = items[idx[i]];
  items.swap(out);
}

// Items in block order; 8x8 tiles are packed four to an item (tiles of equal
// z range only).  Blocks of a class tiled in z-runs (3D, whole blocks) are
// chained along their +z links within `ids` and cut into runs of k blocks;
// one item then takes the same 16x16 tile of each block of a run in turn
// (the default tiling uses runs of two on large classes; see run_len).
// Run items are emitted level by level (the first run of every column, then
// the second, ...), so the workgroups that run at the same time hold
// neighbouring columns at the same height.
void build_items(const hydro_mesh *m, const std::vector<int32_t> &ids, const std::map<int, TileCfg> &cfg,
                 std::vector<WorkItem> &items, int &kmask, std::vector<int32_t> *fused = nullptr) {
  items.clear();
  kmask = 0;
  if (fused) fused->clear();
  std::map<std::pair<int, int>, std::vector<std::array<int, 3>>> pending;
  auto emit8 = [&](std::vector<std::array<int, 3>> &q, int z0, int z1) {
    WorkItem it;
    std::memset(&it, 0, sizeof(it));
    it.kind = hyd::KIND_T8;
    it.z0 = (int16_t)z0;
    it.z1 = (int16_t)z1;
    for (int s = 0; s < 4; ++s) {
      if (s < (int)q.size()) {
        it.block[s] = q[s][0];
        it.x0[s] = (int16_t)q[s][1];
        it.y0[s] = (int16_t)q[s][2];
      } else {
        it.block[s] = -1;
      }
    }
    q.clear();
    items.push_back(it);
    kmask |= 2;
  };
  auto cfg_of = [&](int32_t b) {
    TileCfg c;
    auto f = cfg.find(block_class(m->desc[b], m->ndim));
    if (f != cfg.end()) c = f->second;
    return c;
  };
  // 16x16 tiles per class among the listed blocks (for the default run length)
  std::map<int, int64_t> class_tiles;
  for (int32_t b : ids) {
    const hydro_block_desc &d = m->desc[b];
    class_tiles[block_class(d, m->ndim)] += (int64_t)(d.n[0] / 16) * (d.n[1] / 16);
  }
  // run length of a block: > 1 only for whole-block 16x16 tiling in 3D
  auto run_len = [&](int32_t b) {
    const hydro_block_desc &d = m->desc[b];
    const TileCfg c = cfg_of(b);
    const bool can16 = (d.n[0] % 16 == 0) && (d.n[1] % 16 == 0);
    if (m->ndim != 3 || !can16 || c.tile == 1 || c.tile == 0 || c.tile == TILE_FUSED ||
        (c.zchunk > 0 && c.zchunk < d.n[2]))
      return 1;
    if (c.tile < 0) return default_run(m, class_tiles[block_class(d, m->ndim)]);
    return std::min(c.tile, 4);
  };
  std::unordered_map<int32_t, int> pos;  // position in ids of the blocks tiled in runs
  for (int i = 0; i < (int)ids.size(); ++i)
    if (run_len(ids[i]) > 1) pos[ids[i]] = i;
  for (int32_t b : ids) {
    if (pos.count(b)) continue;
    if (fused && cfg_of(b).tile == TILE_FUSED && fusable(m->desc[b], m->ndim)) {
      fused->push_back(b);  // the fused step takes the whole block
      continue;
    }
    const hydro_block_desc &d = m->desc[b];
    const TileCfg c = cfg_of(b);
    const bool can16 = (d.n[0] % 16 == 0) && (d.n[1] % 16 == 0);
    const bool use16 = can16 && c.tile != 1;
    const int nz = d.n[2];
    const int zc = (m->ndim == 3) ? (c.zchunk > 0 ? std::min(c.zchunk, nz) : nz) : 1;
    for (int z0 = 0; z0 < nz; z0 += zc) {
      const int z1 = std::min(nz, z0 + zc);
      const int T = use16 ? 16 : 8;
      for (int y0 = 0; y0 < d.n[1]; y0 += T)
        for (int x0 = 0; x0 < d.n[0]; x0 += T) {
          if (use16) {
            WorkItem it;
            std::memset(&it, 0, sizeof(it));
            it.kind = hyd::KIND_T16;
            it.block[0] = b;
            it.block[1] = it.block[2] = it.block[3] = -1;
            it.x0[0] = (int16_t)x0;
            it.y0[0] = (int16_t)y0;
            it.z0 = (int16_t)z0;
            it.z1 = (int16_t)z1;
            items.push_back(it);
            kmask |= 1;
          } else {
            auto &q = pending[{z0, z1}];
            q.push_back({b, x0, y0});
            if (q.size() == 4) emit8(q, z0, z1);
          }
        }
    }
  }
  for (auto &kv : pending)
    if (!kv.second.empty()) emit8(kv.second, kv.first.first, kv.first.second);
  if (pos.empty()) {
    order_items(m, items);
    return;
  }

  // z columns of the run-tiled blocks: b -> b' along +z when b' is b's +z
  // neighbour, b is b''s -z neighbour, and both are run-tiled with equal
  // extents and run length
  std::vector<char> taken(ids.size(), 0);
  auto link = [&](int32_t b, int f) -> int32_t {
    const hydro_block_desc &d = m->desc[b];
    if (d.face_kind[f] != HYDRO_NBR) return -1;
    const int32_t o = d.nbr[f];
    auto it = pos.find(o);
    if (it == pos.end() || taken[it->second]) return -1;
    const hydro_block_desc &e = m->desc[o];
    if (e.face_kind[f ^ 1] != HYDRO_NBR || e.nbr[f ^ 1] != b) return -1;
    if (e.n[0] != d.n[0] || e.n[1] != d.n[1] || e.n[2] != d.n[2] || run_len(o) != run_len(b)) return -1;
    return o;
  };
  std::vector<std::vector<std::vector<int32_t>>> levels;  // level -> runs
  for (int32_t b : ids) {
    auto pb = pos.find(b);
    if (pb == pos.end() || taken[pb->second]) continue;
    // head of b's column: walk -z; on a cycle take the member first in ids
    int32_t h = b, first = b;
    for (int32_t p = link(h, 4); p >= 0; p = link(h, 4)) {
      if (p == b) {
        h = first;
        break;
      }
      h = p;
      if (pos[h] < pos[first]) first = h;
    }
    std::vector<int32_t> col;
    for (int32_t c = h; c >= 0; c = link(c, 5)) {
      col.push_back(c);
      taken[pos[c]] = 1;
    }
    const size_t k = (size_t)run_len(b);
    for (size_t r = 0; r * k < col.size(); ++r) {
      if (levels.size() <= r) levels.resize(r + 1);
      levels[r].emplace_back(col.begin() + r * k, col.begin() + std::min(col.size(), (r + 1) * k));
    }
  }
  for (const auto &lv : levels)
    for (const auto &run : lv) {
      const hydro_block_desc &d = m->desc[run[0]];
      for (int y0 = 0; y0 < d.n[1]; y0 += 16)
        for (int x0 = 0; x0 < d.n[0]; x0 += 16) {
          WorkItem it;
          std::memset(&it, 0, sizeof(it));
          it.kind = hyd::KIND_T16;
          for (int s = 0; s < 4; ++s) {
            it.block[s] = s < (int)run.size() ? run[s] : -1;
            it.x0[s] = (int16_t)x0;
            it.y0[s] = (int16_t)y0;
          }
          it.z0 = 0;
          it.z1 = (int16_t)d.n[2];
          items.push_back(it);
          kmask |= 1;
        }
    }
  order_items(m, items);
}

hydro_status upload_items(const std::vector<WorkItem> &items, int kmask, WorkList &wl, hipStream_t s) {
  WorkItem *d = nullptr;
  if (!items.empty()) {
    if (hipMalloc(&d, items.size() * sizeof(WorkItem)) != hipSuccess)
      return fail(HYDRO_ENOMEM, "work list: hipMalloc failed");
    hipError_t e = hipMemcpyAsync(d, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail(HYDRO_EDEVICE, std::string("work list upload: ") + hipGetErrorString(e));
    }
  }
  if (wl.d_items) (void)hipFree(wl.d_items);
  wl.d_items = d;
  wl.nitems = (int)items.size();
  wl.kmask = kmask;
  return HYDRO_OK;
}

hydro_status alloc_time(DevTime **out, hipStream_t s) {
  DevTime *t = nullptr;
  if (hipMalloc(&t, sizeof(DevTime)) != hipSuccess) return fail(HYDRO_ENOMEM, "hipMalloc of time record failed");
  DevTime h;
  std::memset(&h, 0, sizeof(h));
  h.bad_block = INT_MAX;
  hipError_t e = hipMemcpyAsync(t, &h, sizeof(h), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(t);
    return fail(HYDRO_EDEVICE, std::string("time record init: ") + hipGetErrorString(e));
  }
  *out = t;
  return HYDRO_OK;
}

StageArgs stage_args(const hydro_mesh *m, const WorkList &wl, int stage, double dt, const DevTime *dt_dev,
                     DevTime *acc, double gamma, int reset, int remap = 1) {
  StageArgs a;
  a.xcd_remap = remap;
  a.blocks = m->d_blocks;
  a.items = wl.d_items;
  a.nitems = wl.nitems;
  a.reset_time = reset;
  a.src = (stage == 1) ? m->arena : m->u1;
  a.un = m->arena;
  a.dst = (stage == 1) ? m->u1 : m->arena;
  a.dt = dt;
  a.dt_dev = dt_dev;
  a.acc = acc;
  a.gamma = gamma;
  return a;
}

int grid_of(const WorkList &wl, int grid) { return grid > 0 ? std::min(grid, wl.nitems) : wl.nitems; }

// Arguments of the batch's fused-step launch.
hyd::FusedArgs fused_args(const hydro_mesh *m, const int32_t *ids, int n, double *state, double dt,
                          const DevTime *dt_dev, DevTime *acc, double gamma, int rate_only, int remap) {
  hyd::FusedArgs a;
  a.blocks = m->d_blocks;
  a.ids = ids;
  a.nblocks = n;
  a.rate_only = rate_only;
  a.xcd_remap = remap;
  a.state = state;
  a.dt = dt;
  a.dt_dev = dt_dev;
  a.acc = acc;
  a.gamma = gamma;
  return a;
}

// A precision code: HYDRO_FP64 or HYDRO_FP32_FP64 in the low byte, optionally
// with one of HYDRO_SPEEDS_EINFELDT, HYDRO_SPEEDS_PVRS and one of
// HYDRO_RECON_CONSERVED, HYDRO_RECON_CHARACTERISTIC; or HYDRO_FP64 with
// HYDRO_EOS_GAS_RADIATION alone.
bool prec_valid(int32_t p) {
  const int32_t base = p & 0xff, sp = p & (HYDRO_SPEEDS_EINFELDT | HYDRO_SPEEDS_PVRS);
  const int32_t rc = p & (HYDRO_RECON_CONSERVED | HYDRO_RECON_CHARACTERISTIC);
  const int32_t rest = p & ~(0xff | HYDRO_SPEEDS_EINFELDT | HYDRO_SPEEDS_PVRS | HYDRO_RECON_CONSERVED |
                             HYDRO_RECON_CHARACTERISTIC | HYDRO_EOS_GAS_RADIATION);
  if (p & HYDRO_EOS_GAS_RADIATION) return p == (HYDRO_FP64 | HYDRO_EOS_GAS_RADIATION);
  return rest == 0 && sp != (HYDRO_SPEEDS_EINFELDT | HYDRO_SPEEDS_PVRS) &&
         rc != (HYDRO_RECON_CONSERVED | HYDRO_RECON_CHARACTERISTIC) && (base == HYDRO_FP64 || base == HYDRO_FP32_FP64);
}
bool is_mixed(int32_t p) { return (p & 0xff) == HYDRO_FP32_FP64; }
int speeds_of(int32_t p) { return (p & HYDRO_SPEEDS_EINFELDT) ? 1 : (p & HYDRO_SPEEDS_PVRS) ? 2 : 0; }
int recon_of(int32_t p) { return (p & HYDRO_RECON_CONSERVED) ? 1 : (p & HYDRO_RECON_CHARACTERISTIC) ? 2 : 0; }
int eos_of(int32_t p) { return (p & HYDRO_EOS_GAS_RADIATION) ? 1 : 0; }

// Workgroups of the batch's fused-step launch: as many as can be resident
// (three per CU for the mixed kernel, two for the FP64 one, whose LDS and
// registers allow no more), each looping over its share of the blocks and
// loading the next block while it computes the current one.
int fused_grid(const hydro_batch *b) {
  const int resident = (is_mixed(b->prec) ? 3 : 2) * std::max(b->m->num_cu, 1);
  return std::min(b->nfused, resident);
}


hydro_status launch_stage_wl(const hydro_mesh *m, int prec, int stage, const WorkList &wl, int grid,
                             hipStream_t s, const StageArgs &a, int occ = 0) {
  hipError_t e = hyd::launch_stage(m->ndim, is_mixed(prec), stage, wl.kmask, speeds_of(prec), recon_of(prec),
                                   eos_of(prec), grid_of(wl, grid), s, a, occ);
  if (e != hipSuccess) return fail(HYDRO_EDEVICE, std::string("stage launch: ") + hipGetErrorString(e));
  return HYDRO_OK;
}

hydro_status read_time(const hydro_mesh *m, const DevTime *d, DevTime &h) {
  HIP_TRY(hipMemcpyAsync(&h, d, sizeof(DevTime), hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return HYDRO_OK;
}

hydro_status nonphys(const DevTime &h) {
  return fail(HYDRO_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or non-finite)" +
                                  (h.bad_block != INT_MAX ? " in block " + std::to_string(h.bad_block) : std::string()));
}

// The batch's work list and fused-block list from its tiling settings, all
// or nothing: on an error the batch keeps its previous lists.
hydro_status rebuild_batch_items(hydro_batch *b) {
  std::vector<WorkItem> items;
  std::vector<int32_t> fused;
  int kmask = 0;
  build_items(b->m, b->ids, b->cfg, items, kmask, &fused);
  int32_t *d = nullptr;
  if (!fused.empty()) {
    if (hipMalloc(&d, fused.size() * sizeof(int32_t)) != hipSuccess)
      return fail(HYDRO_ENOMEM, "fused block list: hipMalloc failed");
    hipError_t e = hipMemcpyAsync(d, fused.data(), fused.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  b->m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->m->stream);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail(HYDRO_EDEVICE, std::string("fused block list upload: ") + hipGetErrorString(e));
    }
  }
  WorkList wl;
  hydro_status st = upload_items(items, kmask, wl, b->m->stream);
  if (st) {
    if (d) (void)hipFree(d);
    return st;
  }
  if (b->wl.d_items) (void)hipFree(b->wl.d_items);
  b->wl = wl;
  if (b->d_fused) (void)hipFree(b->d_fused);
  b->d_fused = d;
  b->nfused = (int)fused.size();
  // the captured graph holds the old work list
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  return HYDRO_OK;
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char *hydro_last_error(void) { return g_err; }

hydro_status hydro_mesh_create(const hydro_block_desc *blocks, int32_t nblocks, int32_t ndim, double *arena,
                               int64_t arena_len, void *stream, hydro_mesh **out) {
  if (!out) return fail(HYDRO_EINVAL, "mesh: out is null");
  *out = nullptr;
  hydro_status st = validate_mesh(blocks, nblocks, ndim, arena, arena_len);
  if (st) return st;

  hydro_mesh *m = new hydro_mesh();
  m->ndim = ndim;
  m->nblocks = nblocks;
  m->arena = arena;
  m->arena_len = arena_len;
  m->stream = (hipStream_t)stream;
  m->desc.assign(blocks, blocks + nblocks);
  std::vector<DevBlock> hb(nblocks);
  for (int b = 0; b < nblocks; ++b) hb[b] = make_devblock(blocks, b, ndim);

  auto cleanup = [&](hydro_status s, const std::string &msg) {
    if (m->u1) (void)hipFree(m->u1);
    if (m->d_blocks) (void)hipFree(m->d_blocks);
    delete m;
    return fail(s, msg);
  };
  if (hipGetDevice(&m->device) != hipSuccess) return cleanup(HYDRO_EDEVICE, "mesh: no HIP device");
  if (hipDeviceGetAttribute(&m->num_cu, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess)
    return cleanup(HYDRO_EDEVICE, "mesh: device query failed");
  if (hipMalloc(&m->u1, (size_t)arena_len * sizeof(double)) != hipSuccess)
    return cleanup(HYDRO_ENOMEM, "mesh: hipMalloc of the stage buffer failed");
  if (hipMalloc(&m->d_blocks, (size_t)nblocks * sizeof(DevBlock)) != hipSuccess)
    return cleanup(HYDRO_ENOMEM, "mesh: hipMalloc of the block table failed");
  hipError_t e = hipMemcpyAsync(m->d_blocks, hb.data(), hb.size() * sizeof(DevBlock), hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return cleanup(HYDRO_EDEVICE, std::string("mesh: block table upload: ") + hipGetErrorString(e));
  *out = m;
  return HYDRO_OK;
}

hydro_status hydro_mesh_destroy(hydro_mesh *m) {
  if (!m) return fail(HYDRO_EINVAL, "mesh is null");
  if (m->children) return fail(HYDRO_ESTATE, "mesh still has packets or batches");
  (void)hipStreamSynchronize(m->stream);
  (void)hipFree(m->u1);
  (void)hipFree(m->d_blocks);
  delete m;
  return HYDRO_OK;
}

hydro_status hydro_packet_create(hydro_mesh *m, const int32_t *block_ids, int32_t nblocks, int32_t precision,
                                 hydro_packet **out) {
  if (!out) return fail(HYDRO_EINVAL, "packet: out is null");
  *out = nullptr;
  if (!m) return fail(HYDRO_EINVAL, "packet: mesh is null");
  if (!block_ids || nblocks <= 0) return fail(HYDRO_EINVAL, "packet: need at least one block id");
  if (!prec_valid(precision)) return fail(HYDRO_EINVAL, "packet: bad precision");
  std::vector<char> seen(m->nblocks, 0);
  for (int i = 0; i < nblocks; ++i) {
    const int b = block_ids[i];
    if (b < 0 || b >= m->nblocks) return fail(HYDRO_EINVAL, "packet: block id out of range");
    if (seen[b]) return fail(HYDRO_EINVAL, "packet: duplicate block id " + std::to_string(b));
    seen[b] = 1;
  }
  hydro_packet *p = new hydro_packet();
  p->m = m;
  p->ids.assign(block_ids, block_ids + nblocks);
  p->prec = precision;
  p->closed = true;
  for (int b : p->ids)
    for (int f = 0; f < 2 * m->ndim; ++f)
      if (m->desc[b].face_kind[f] == HYDRO_NBR && !seen[m->desc[b].nbr[f]]) p->closed = false;
  std::vector<WorkItem> items;
  int kmask = 0;
  build_items(m, p->ids, {}, items, kmask);
  hydro_status st = upload_items(items, kmask, p->wl, m->stream);
  if (!st) st = alloc_time(&p->d_time, m->stream);
  if (st) {
    if (p->wl.d_items) (void)hipFree(p->wl.d_items);
    delete p;
    return st;
  }
  m->children++;
  *out = p;
  return HYDRO_OK;
}

hydro_status hydro_packet_destroy(hydro_packet *p) {
  if (!p) return fail(HYDRO_EINVAL, "packet is null");
  if (p->batches) return fail(HYDRO_ESTATE, "packet is still part of a batch");
  (void)hipStreamSynchronize(p->m->stream);
  (void)hipFree(p->wl.d_items);
  (void)hipFree(p->d_time);
  p->m->children--;
  delete p;
  return HYDRO_OK;
}

static hydro_status check_step_args(double dt, double gamma) {
  if (!finite_pos(dt)) return fail(HYDRO_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(gamma) || gamma <= 1.0) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  return HYDRO_OK;
}

hydro_status hydro_packet_advance(hydro_packet *p, double dt, double gamma) {
  if (!p) return fail(HYDRO_EINVAL, "packet is null");
  hydro_status st = check_step_args(dt, gamma);
  if (st) return st;
  if (!p->closed)
    return fail(HYDRO_ESTATE, "packet is not closed under its NBR links; use a batch to keep stages synchronous");
  hydro_mesh *m = p->m;
  const int prec = p->prec;
  p->lam_valid = false;
  st = launch_stage_wl(m, prec, 1, p->wl, 0, m->stream, stage_args(m, p->wl, 1, dt, nullptr, p->d_time, gamma, 1));
  if (st) return st;
  st = launch_stage_wl(m, prec, 2, p->wl, 0, m->stream, stage_args(m, p->wl, 2, dt, nullptr, p->d_time, gamma, 0));
  if (st) return st;
  p->lam_valid = true;
  p->lam_gamma = gamma;
  return HYDRO_OK;
}

hydro_status hydro_packet_reduce_dt(hydro_packet *p, double gamma, double cfl, double *dt_out) {
  if (!p || !dt_out) return fail(HYDRO_EINVAL, "packet and dt_out must be non-null");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
  if (!std::isfinite(gamma) || gamma <= 1.0) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  hydro_mesh *m = p->m;
  if (!(p->lam_valid && p->lam_gamma == gamma)) {
    hipError_t e = hyd::launch_reset(p->d_time, m->stream);
    if (e == hipSuccess)
      e = hyd::launch_lambda(m->ndim, is_mixed(p->prec), p->wl.kmask, eos_of(p->prec), p->wl.nitems, m->stream,
                             stage_args(m, p->wl, 1, 0.0, nullptr, p->d_time, gamma, 0));
    if (e != hipSuccess) return fail(HYDRO_EDEVICE, std::string("rate launch: ") + hipGetErrorString(e));
  }
  DevTime h;
  hydro_status st = read_time(m, p->d_time, h);
  if (st) return st;
  if (h.status) return nonphys(h);
  const double lam = [&] {
    double d;
    std::memcpy(&d, &h.lam_bits, sizeof(d));
    return d;
  }();
  if (!(lam > 0.0)) return fail(HYDRO_ENONPHYS, "CFL rate is zero or invalid");
  *dt_out = cfl / lam;
  p->lam_valid = true;
  p->lam_gamma = gamma;
  return HYDRO_OK;
}

hydro_status hydro_batch_create(hydro_packet *const *packets, int32_t npackets, hydro_batch **out) {
  if (!out) return fail(HYDRO_EINVAL, "batch: out is null");
  *out = nullptr;
  if (!packets || npackets <= 0) return fail(HYDRO_EINVAL, "batch: need at least one packet");
  hydro_mesh *m = packets[0] ? packets[0]->m : nullptr;
  if (!m) return fail(HYDRO_EINVAL, "batch: null packet");
  const int prec = packets[0]->prec;
  std::vector<char> seen(m->nblocks, 0);
  std::vector<int32_t> ids;
  for (int i = 0; i < npackets; ++i) {
    const hydro_packet *p = packets[i];
    if (!p || p->m != m) return fail(HYDRO_EINVAL, "batch: packets must share one mesh");
    if (p->prec != prec) return fail(HYDRO_EINVAL, "batch: packets must share one precision");
    for (int b : p->ids) {
      if (seen[b]) return fail(HYDRO_EINVAL, "batch: block " + std::to_string(b) + " is in two packets");
      seen[b] = 1;
      ids.push_back(b);
    }
  }
  hydro_batch *bt = new hydro_batch();
  bt->m = m;
  bt->packets.assign(packets, packets + npackets);
  bt->ids = std::move(ids);
  bt->prec = prec;
  // XCD renumbering pays where neighbouring blocks read each other's cells;
  // blocks that link to none gain nothing from sharing an L2, and contiguous
  // spans of uneven items would load the XCDs unevenly
  bool linked = false;
  for (int b : bt->ids)
    for (int f = 0; f < 2 * m->ndim; ++f) linked = linked || m->desc[b].face_kind[f] == HYDRO_NBR;
  bt->remap = linked ? 1 : 0;
  hydro_status st = rebuild_batch_items(bt);
  if (!st) st = alloc_time(&bt->d_time, m->stream);
  if (!st && (hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking) != hipSuccess ||
              hipStreamCreateWithFlags(&bt->side_stream, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&bt->fork_ev, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&bt->join_ev, hipEventDisableTiming) != hipSuccess))
    st = fail(HYDRO_EDEVICE, "batch: stream or event creation failed");
  if (st) {
    if (bt->fork_ev) (void)hipEventDestroy(bt->fork_ev);
    if (bt->join_ev) (void)hipEventDestroy(bt->join_ev);
    if (bt->side_stream) (void)hipStreamDestroy(bt->side_stream);
    if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
    if (bt->wl.d_items) (void)hipFree(bt->wl.d_items);
    if (bt->d_fused) (void)hipFree(bt->d_fused);
    if (bt->d_time) (void)hipFree(bt->d_time);
    delete bt;
    return st;
  }
  for (auto *p : bt->packets) p->batches++;
  m->children++;
  *out = bt;
  return HYDRO_OK;
}

hydro_status hydro_batch_destroy(hydro_batch *b) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  (void)hipStreamSynchronize(b->m->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->join_ev) (void)hipEventDestroy(b->join_ev);
  (void)hipFree(b->wl.d_items);
  if (b->d_fused) (void)hipFree(b->d_fused);
  (void)hipFree(b->d_time);
  for (auto *p : b->packets) p->batches--;
  b->m->children--;
  delete b;
  return HYDRO_OK;
}

hydro_status hydro_batch_advance_plain(hydro_batch *b, double dt, double gamma) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  hydro_status st = check_step_args(dt, gamma);
  if (st) return st;
  hydro_mesh *m = b->m;
  const int prec = b->prec;
  for (auto *p : b->packets) {
    p->lam_valid = false;
    st = launch_stage_wl(m, prec, 1, p->wl, 0, m->stream, stage_args(m, p->wl, 1, dt, nullptr, p->d_time, gamma, 1));
    if (st) return st;
  }
  for (auto *p : b->packets) {
    st = launch_stage_wl(m, prec, 2, p->wl, 0, m->stream, stage_args(m, p->wl, 2, dt, nullptr, p->d_time, gamma, 0));
    if (st) return st;
    p->lam_valid = true;
    p->lam_gamma = gamma;
  }
  return HYDRO_OK;
}

static hydro_status capture_step(hydro_batch *b, double cfl, double gamma) {
  hydro_mesh *m = b->m;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  const int prec = b->prec;
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hydro_status st = HYDRO_OK;
  // The fused blocks share no cells with the others, so their launch is a
  // branch of the graph beside the two stage launches (both branches fold
  // their CFL rate into the accumulator with atomics); the dt update waits
  // for both.
  if (b->nfused > 0) {
    if (hipEventRecord(b->fork_ev, b->cap_stream) != hipSuccess ||
        hipStreamWaitEvent(b->side_stream, b->fork_ev, 0) != hipSuccess ||
        hyd::launch_fused(is_mixed(prec), fused_grid(b), b->side_stream,
                          fused_args(m, b->d_fused, b->nfused, m->arena, 0.0, b->d_time, b->d_time, gamma, 0,
                                     b->remap)) != hipSuccess ||
        hipEventRecord(b->join_ev, b->side_stream) != hipSuccess)
      st = fail(HYDRO_EDEVICE, "fused step branch capture failed");
  }
  if (!st)
    st = launch_stage_wl(m, prec, 1, b->wl, b->grid, b->cap_stream,
                         stage_args(m, b->wl, 1, 0.0, b->d_time, b->d_time, gamma, 0, b->remap), b->occ);
  if (!st)
    st = launch_stage_wl(m, prec, 2, b->wl, b->grid, b->cap_stream,
                         stage_args(m, b->wl, 2, 0.0, b->d_time, b->d_time, gamma, 0, b->remap), b->occ);
  if (!st && b->nfused > 0 && hipStreamWaitEvent(b->cap_stream, b->join_ev, 0) != hipSuccess)
    st = fail(HYDRO_EDEVICE, "fused step branch join failed");
  if (!st && hyd::launch_finalize(b->d_time, cfl, 0, b->cap_stream) != hipSuccess)
    st = fail(HYDRO_EDEVICE, "finalize launch failed");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(HYDRO_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(HYDRO_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  b->graph = g;
  b->g_cfl = cfl;
  b->g_gamma = gamma;
  return HYDRO_OK;
}

}  // extern "C"

// nsteps graph replays; with step_ms, HIP events on the mesh stream around
// every replay give each step's device time.
static hydro_status batch_run(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *t_out,
                              double *step_ms) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  if (nsteps < 0) return fail(HYDRO_EINVAL, "nsteps must be >= 0");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
  if (!std::isfinite(gamma) || gamma <= 1.0) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  hydro_mesh *m = b->m;
  if (!b->gexec || b->g_cfl != cfl || b->g_gamma != gamma) {
    hydro_status st = capture_step(b, cfl, gamma);
    if (st) return st;
  }
  for (auto *p : b->packets) p->lam_valid = false;
  // dt of the first step from the current state
  hipError_t e = hyd::launch_reset(b->d_time, m->stream);
  if (e == hipSuccess)
    e = hyd::launch_lambda(m->ndim, is_mixed(b->prec), b->wl.kmask, eos_of(b->prec), grid_of(b->wl, b->grid), m->stream,
                           stage_args(m, b->wl, 1, 0.0, nullptr, b->d_time, gamma, 0, b->remap));
  if (e == hipSuccess)
    e = hyd::launch_fused(is_mixed(b->prec), fused_grid(b), m->stream,
                          fused_args(m, b->d_fused, b->nfused, m->arena, 0.0, nullptr, b->d_time, gamma, 1, b->remap));
  if (e == hipSuccess) e = hyd::launch_finalize(b->d_time, cfl, 1, m->stream);
  if (e != hipSuccess) return fail(HYDRO_EDEVICE, std::string("batch run setup: ") + hipGetErrorString(e));
  std::vector<hipEvent_t> ev(step_ms ? nsteps + 1 : 0, nullptr);
  hydro_status st = HYDRO_OK;
  for (auto &x : ev)
    if (!st && hipEventCreate(&x) != hipSuccess) st = fail(HYDRO_EDEVICE, "event create");
  if (!st && step_ms && hipEventRecord(ev[0], m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "event record");
  for (int s = 0; s < nsteps && !st; ++s) {
    if (hipGraphLaunch(b->gexec, m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "graph launch");
    if (!st && step_ms && hipEventRecord(ev[s + 1], m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "event record");
  }
  DevTime h;
  if (!st) st = read_time(m, b->d_time, h);  // synchronises the mesh stream
  for (int s = 0; s < nsteps && !st && step_ms; ++s) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev[s], ev[s + 1]) != hipSuccess) st = fail(HYDRO_EDEVICE, "event time");
    step_ms[s] = ms;
  }
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st) return st;
  // after a failure t is the time at the end of the failing step (later
  // replays left the state and t alone)
  if (t_out) *t_out = h.t;
  if (h.status) return nonphys(h);
  return HYDRO_OK;
}

extern "C" {

hydro_status hydro_batch_run(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *t_out) {
  return batch_run(b, nsteps, cfl, gamma, t_out, nullptr);
}

hydro_status hydro_batch_run_timed(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *t_out,
                                   double *step_ms) {
  if (!step_ms) return fail(HYDRO_EINVAL, "step_ms must be non-null");
  return batch_run(b, nsteps, cfl, gamma, t_out, step_ms);
}

hydro_status hydro_batch_time_kernels(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *ms_out) {
  if (!b || !ms_out) return fail(HYDRO_EINVAL, "batch and ms_out must be non-null");
  if (nsteps < 1) return fail(HYDRO_EINVAL, "nsteps must be >= 1");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
  if (!std::isfinite(gamma) || gamma <= 1.0) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  hydro_mesh *m = b->m;
  const int prec = b->prec;
  for (auto *p : b->packets) p->lam_valid = false;
  hipError_t e = hyd::launch_reset(b->d_time, m->stream);
  if (e == hipSuccess)
    e = hyd::launch_lambda(m->ndim, is_mixed(prec), b->wl.kmask, eos_of(prec), grid_of(b->wl, b->grid), m->stream,
                           stage_args(m, b->wl, 1, 0.0, nullptr, b->d_time, gamma, 0, b->remap));
  if (e == hipSuccess)
    e = hyd::launch_fused(is_mixed(prec), fused_grid(b), m->stream,
                          fused_args(m, b->d_fused, b->nfused, m->arena, 0.0, nullptr, b->d_time, gamma, 1, b->remap));
  if (e == hipSuccess) e = hyd::launch_finalize(b->d_time, cfl, 1, m->stream);
  if (e != hipSuccess) return fail(HYDRO_EDEVICE, std::string("timing setup: ") + hipGetErrorString(e));
  std::vector<hipEvent_t> ev(3 * nsteps + 1, nullptr);
  hydro_status st = HYDRO_OK;
  for (auto &x : ev)
    if (!st && hipEventCreate(&x) != hipSuccess) st = fail(HYDRO_EDEVICE, "event create");
  if (!st && hipEventRecord(ev[0], m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "event record");
  for (int s = 0; s < nsteps && !st; ++s) {
    st = launch_stage_wl(m, prec, 1, b->wl, b->grid, m->stream,
                         stage_args(m, b->wl, 1, 0.0, b->d_time, b->d_time, gamma, 0, b->remap), b->occ);
    if (!st && hipEventRecord(ev[3 * s + 1], m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "event record");
    if (!st)
      st = launch_stage_wl(m, prec, 2, b->wl, b->grid, m->stream,
                           stage_args(m, b->wl, 2, 0.0, b->d_time, b->d_time, gamma, 0, b->remap), b->occ);
    if (!st && hyd::launch_fused(is_mixed(prec), fused_grid(b), m->stream,
                                 fused_args(m, b->d_fused, b->nfused, m->arena, 0.0, b->d_time, b->d_time, gamma, 0,
                                            b->remap)) != hipSuccess)
      st = fail(HYDRO_EDEVICE, "fused step launch failed");
    if (!st && hipEventRecord(ev[3 * s + 2], m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "event record");
    if (!st && hyd::launch_finalize(b->d_time, cfl, 0, m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "finalize");
    if (!st && hipEventRecord(ev[3 * s + 3], m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "event record");
  }
  if (!st && hipEventSynchronize(ev[3 * nsteps]) != hipSuccess) st = fail(HYDRO_EDEVICE, "event sync");
  double t1 = 0, t2 = 0, tall = 0;
  for (int s = 0; s < nsteps && !st; ++s) {
    float a = 0, c = 0, d = 0;
    (void)hipEventElapsedTime(&a, ev[3 * s], ev[3 * s + 1]);
    (void)hipEventElapsedTime(&c, ev[3 * s + 1], ev[3 * s + 2]);
    (void)hipEventElapsedTime(&d, ev[3 * s], ev[3 * s + 3]);
    t1 += a;
    t2 += c;
    tall += d;
  }
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st) return st;
  DevTime h;
  st = read_time(m, b->d_time, h);
  if (st) return st;
  if (h.status) return nonphys(h);
  ms_out[0] = t1 / nsteps;
  ms_out[1] = t2 / nsteps;
  ms_out[2] = tall / nsteps;
  return HYDRO_OK;
}

}  // extern "C"

// ------------------------------------------------------- host-resident packets
struct hydro_stream {
  int ndim = 3;
  int prec = HYDRO_FP64;
  int device = 0;
  double *host = nullptr;
  std::vector<hydro_block_desc> desc;
  std::vector<int32_t> pstart;     // npackets + 1
  std::vector<int64_t> phost;      // host element offset of each packet
  std::vector<int64_t> plen;       // elements of each packet
  // Transfer units: runs of consecutive GPU packets, adjacent in the arena,
  // that a slot copies in, advances and copies back as one (each at least
  // unit_bytes long, or a single packet when unit_bytes is 0)
  int64_t unit_bytes = 0;
  std::vector<int32_t> ustart;     // first packet of each unit, nunits + 1 entries
  std::vector<int64_t> uhost;      // host element offset of each unit
  std::vector<int64_t> ulen;       // elements of each unit
  std::vector<WorkList> wl;        // per unit, block ids into the shared table
  std::vector<int> uslot;          // slot of each unit: the least loaded so far, in unit order
  int64_t slot_len = 0;            // elements each slot buffer holds
  DevBlock *d_blocks = nullptr;    // offsets relative to the first element of the block's unit
  struct Slot {
    hipStream_t stream = nullptr;
    double *state = nullptr;
    double *u1 = nullptr;
    hipEvent_t done = nullptr;
  };
  std::vector<Slot> slots;
  hipStream_t ctl = nullptr;
  hipEvent_t ready = nullptr;
  DevTime *d_time = nullptr;
  // CPU/GPU split: the last cpu_packets packets are advanced by host threads
  int cpu_packets = 0;
  int cpu_threads = 1;
  std::vector<double> cpu_u1;  // first-stage state of the CPU packets (host)
  std::vector<int32_t> cpu_ids;
  std::vector<double *> cpu_un;        // per block (global id): Un in the host arena
  std::vector<double *> cpu_u1p;       // per block: its first-stage state in cpu_u1
};

namespace {

void stream_free(hydro_stream *s) {
  for (auto &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.state) (void)hipFree(sl.state);
    if (sl.u1) (void)hipFree(sl.u1);
  }
  for (auto &w : s->wl)
    if (w.d_items) (void)hipFree(w.d_items);
  if (s->ready) (void)hipEventDestroy(s->ready);
  if (s->ctl) (void)hipStreamDestroy(s->ctl);
  if (s->d_blocks) (void)hipFree(s->d_blocks);
  if (s->d_time) (void)hipFree(s->d_time);
  delete s;
}

// Units of uneven size: each unit goes to the slot with the fewest bytes so
// far, so the slot streams finish a step together.
void assign_slots(hydro_stream *s) {
  std::vector<int64_t> load(s->slots.size(), 0);
  s->uslot.assign(s->ulen.size(), -1);
  for (size_t u = 0; u < s->ulen.size(); ++u) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    s->uslot[u] = k;
    load[k] += s->ulen[u];
  }
}

// The GPU packets [0, npackets - cpu_packets) cut into transfer units of at
// least unit_bytes; the block table (offsets relative to each block's unit),
// the units' work lists and, where a unit outgrows them, the slot buffers
// follow.  All or nothing: on an error the stream keeps its previous units,
// buffers and table, and the caller keeps its previous settings.
hydro_status build_units(hydro_stream *s, int64_t unit_bytes, int cpu_packets) {
  const int np = (int)s->pstart.size() - 1, ngpu = np - cpu_packets;
  const int nblocks = (int)s->desc.size();
  std::vector<int32_t> ustart;
  std::vector<int64_t> uhost, ulen;
  for (int p = 0; p < ngpu;) {
    int q = p + 1;
    int64_t len = s->plen[p];
    while (q < ngpu && len * (int64_t)sizeof(double) < unit_bytes && s->phost[q] == s->phost[p] + len)
      len += s->plen[q++];
    ustart.push_back(p);
    uhost.push_back(s->phost[p]);
    ulen.push_back(len);
    p = q;
  }
  ustart.push_back(ngpu);
  const int nu = (int)ulen.size();
  // new work lists and, if needed, larger slot buffers, before anything is replaced
  std::vector<WorkList> wl(nu);
  std::vector<std::pair<double *, double *>> bufs;
  auto drop = [&]() {
    for (auto &w : wl)
      if (w.d_items) (void)hipFree(w.d_items);
    for (auto &pr : bufs) {
      if (pr.first) (void)hipFree(pr.first);
      if (pr.second) (void)hipFree(pr.second);
    }
  };
  hydro_mesh view;  // descriptors only, for the item builder
  view.ndim = s->ndim;
  view.nblocks = nblocks;
  view.desc = s->desc;
  for (int u = 0; u < nu; ++u) {
    std::vector<int32_t> ids;
    for (int b = s->pstart[ustart[u]]; b < s->pstart[ustart[u + 1]]; ++b) ids.push_back(b);
    std::vector<WorkItem> items;
    int kmask = 0;
    build_items(&view, ids, {}, items, kmask);
    hydro_status st = upload_items(items, kmask, wl[u], s->ctl);
    if (st) {
      drop();
      return st;
    }
  }
  int64_t maxlen = 0;
  for (int64_t l : ulen) maxlen = std::max(maxlen, l);
  if (maxlen > s->slot_len) {
    bufs.assign(s->slots.size(), {nullptr, nullptr});
    for (auto &pr : bufs)
      if (hipMalloc(&pr.first, (size_t)maxlen * sizeof(double)) != hipSuccess ||
          hipMalloc(&pr.second, (size_t)maxlen * sizeof(double)) != hipSuccess) {
        drop();
        return fail(HYDRO_ENOMEM, "stream: hipMalloc of a staging slot failed");
      }
  }
  std::vector<hydro_block_desc> local(s->desc);
  for (int u = 0; u < nu; ++u)
    for (int b = s->pstart[ustart[u]]; b < s->pstart[ustart[u + 1]]; ++b) local[b].offset -= uhost[u];
  std::vector<DevBlock> hb(nblocks);
  for (int b = 0; b < nblocks; ++b) hb[b] = make_devblock(local.data(), b, s->ndim);
  for (auto &sl : s->slots)  // no copy or launch of the old set-up may still use the table
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  if (hipMemcpyAsync(s->d_blocks, hb.data(), hb.size() * sizeof(DevBlock), hipMemcpyHostToDevice, s->ctl) !=
          hipSuccess ||
      hipStreamSynchronize(s->ctl) != hipSuccess) {
    drop();
    return fail(HYDRO_EDEVICE, "stream: block table upload failed");
  }
  // commit
  for (auto &w : s->wl)
    if (w.d_items) (void)hipFree(w.d_items);
  s->wl.swap(wl);
  if (!bufs.empty()) {
    for (size_t k = 0; k < s->slots.size(); ++k) {
      auto &sl = s->slots[k];
      if (sl.state) (void)hipFree(sl.state);
      if (sl.u1) (void)hipFree(sl.u1);
      sl.state = bufs[k].first;
      sl.u1 = bufs[k].second;
    }
    s->slot_len = maxlen;
  }
  s->ustart.swap(ustart);
  s->uhost.swap(uhost);
  s->ulen.swap(ulen);
  s->unit_bytes = unit_bytes;
  assign_slots(s);
  return HYDRO_OK;
}

StageArgs slot_args(const hydro_stream *s, const hydro_stream::Slot &sl, const WorkList &wl, int stage, double gamma) {
  StageArgs a;
  a.blocks = s->d_blocks;
  a.items = wl.d_items;
  a.nitems = wl.nitems;
  a.reset_time = 0;
  a.xcd_remap = 1;
  a.src = (stage == 1) ? sl.state : sl.u1;
  a.un = sl.state;
  a.dst = (stage == 1) ? sl.u1 : sl.state;
  a.dt = 0.0;
  a.dt_dev = s->d_time;
  a.acc = s->d_time;
  a.gamma = gamma;
  return a;
}

}  // namespace

extern "C" {

hydro_status hydro_stream_create(const hydro_block_desc *blocks, int32_t nblocks, int32_t ndim, double *host_arena,
                                 int64_t arena_len, const int32_t *packet_start, int32_t npackets,
                                 int32_t precision, int32_t nslots, hydro_stream **out) {
  if (!out) return fail(HYDRO_EINVAL, "stream: out is null");
  *out = nullptr;
  hydro_status st = validate_mesh(blocks, nblocks, ndim, host_arena, arena_len);
  if (st) return st;
  if (!prec_valid(precision)) return fail(HYDRO_EINVAL, "stream: bad precision");
  if (nslots < 1 || nslots > 16) return fail(HYDRO_EINVAL, "stream: nslots must be in 1..16");
  if (!packet_start || npackets < 1) return fail(HYDRO_EINVAL, "stream: need at least one packet");
  if (packet_start[0] != 0 || packet_start[npackets] != nblocks)
    return fail(HYDRO_EINVAL, "stream: packet ranges must start at 0 and end at nblocks");
  for (int p = 0; p < npackets; ++p)
    if (packet_start[p + 1] <= packet_start[p]) return fail(HYDRO_EINVAL, "stream: empty or decreasing packet range");
  std::vector<int64_t> phost(npackets), plen(npackets);
  for (int p = 0; p < npackets; ++p) {
    const int b0 = packet_start[p], b1 = packet_start[p + 1];
    int64_t end = blocks[b0].offset;
    for (int b = b0; b < b1; ++b) {
      if (blocks[b].offset != end)
        return fail(HYDRO_EINVAL, "stream: blocks of packet " + std::to_string(p) + " are not contiguous in the arena");
      end += 5 * (int64_t)blocks[b].n[0] * blocks[b].n[1] * blocks[b].n[2];
      for (int f = 0; f < 2 * ndim; ++f)
        if (blocks[b].face_kind[f] == HYDRO_NBR && (blocks[b].nbr[f] < b0 || blocks[b].nbr[f] >= b1))
          return fail(HYDRO_EINVAL, "stream: packet " + std::to_string(p) + " is not closed (block " +
                                        std::to_string(b) + " links outside it)");
    }
    phost[p] = blocks[b0].offset;
    plen[p] = end - blocks[b0].offset;
  }

  hydro_stream *s = new hydro_stream();
  s->ndim = ndim;
  s->prec = precision;
  s->host = host_arena;
  s->desc.assign(blocks, blocks + nblocks);
  s->pstart.assign(packet_start, packet_start + npackets + 1);
  s->phost = phost;
  s->plen = plen;
  auto bail = [&](hydro_status e, const std::string &msg) {
    stream_free(s);
    return fail(e, msg);
  };
  if (hipGetDevice(&s->device) != hipSuccess) return bail(HYDRO_EDEVICE, "stream: no HIP device");
  if (hipStreamCreateWithFlags(&s->ctl, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->ready, hipEventDisableTiming) != hipSuccess)
    return bail(HYDRO_EDEVICE, "stream: control stream creation failed");
  if (hipMalloc(&s->d_blocks, (size_t)nblocks * sizeof(DevBlock)) != hipSuccess)
    return bail(HYDRO_ENOMEM, "stream: hipMalloc of the block table failed");
  if (alloc_time(&s->d_time, s->ctl)) return bail(HYDRO_ENOMEM, "stream: time record allocation failed");
  s->slots.resize(nslots);
  for (auto &sl : s->slots)
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
      return bail(HYDRO_EDEVICE, "stream: slot stream creation failed");
  st = build_units(s, 0, 0);  // one packet per unit; allocates the slot buffers
  if (st) {
    stream_free(s);
    return st;
  }
  *out = s;
  return HYDRO_OK;
}

hydro_status hydro_stream_destroy(hydro_stream *s) {
  if (!s) return fail(HYDRO_EINVAL, "stream is null");
  stream_free(s);
  return HYDRO_OK;
}

hydro_status hydro_stream_run(hydro_stream *s, int32_t nsteps, double cfl, double gamma, double *t_out) {
  if (!s) return fail(HYDRO_EINVAL, "stream is null");
  if (nsteps < 0) return fail(HYDRO_EINVAL, "nsteps must be >= 0");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
  if (!std::isfinite(gamma) || gamma <= 1.0) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  const int nu = (int)s->ulen.size();  // GPU transfer units; packets past them run on the host
  const bool split = s->cpu_packets > 0;
  const int prec = s->prec;
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  bool good = true;
  const int ns = (int)s->slots.size();
  std::vector<int> lastu(ns, -1);  // last unit of each slot
  for (int u = 0; u < nu; ++u) lastu[s->uslot[u]] = u;
  // every slot stream starts after the control stream's last work
  auto fan_out = [&]() {
    good = good && ok(hipEventRecord(s->ready, s->ctl));
    for (auto &sl : s->slots) good = good && ok(hipStreamWaitEvent(sl.stream, s->ready, 0));
  };
  auto done = [&](hydro_stream::Slot &sl) {  // the control stream waits for this slot's work so far
    good = good && ok(hipEventRecord(sl.done, sl.stream));
    good = good && ok(hipStreamWaitEvent(s->ctl, sl.done, 0));
  };
  auto copy_in = [&](int u, hydro_stream::Slot &sl) {
    good = good && ok(hipMemcpyAsync(sl.state, s->host + s->uhost[u], (size_t)s->ulen[u] * sizeof(double),
                                     hipMemcpyHostToDevice, sl.stream));
  };
  // the host share: its CFL rate and non-physical flag go into the device
  // accumulator on the control stream, ahead of the dt update
  auto fold = [&](const hyd::HostRate &r) {
    good = good && ok(hyd::launch_fold(s->d_time, r.lam, r.bad, r.bad_block, s->ctl));
  };
  hyd::HostStage H;
  H.desc = s->desc.data();
  H.ndim = s->ndim;
  H.ids = s->cpu_ids;
  H.gamma = gamma;
  // dt of the first step: rate of every packet's current state
  good = good && ok(hyd::launch_reset(s->d_time, s->ctl));
  fan_out();
  for (int u = 0; u < nu && good; ++u) {
    auto &sl = s->slots[s->uslot[u]];
    copy_in(u, sl);
    good = good && ok(hyd::launch_lambda(s->ndim, is_mixed(prec), s->wl[u].kmask, eos_of(prec), s->wl[u].nitems, sl.stream,
                                         slot_args(s, sl, s->wl[u], 1, gamma)));
    if (u == lastu[s->uslot[u]]) done(sl);
  }
  if (split && good) {
    H.src = s->cpu_un.data();
    fold(hyd::host_run(H, s->cpu_threads, true));
  }
  good = good && ok(hyd::launch_finalize(s->d_time, cfl, 1, s->ctl));
  good = good && ok(hipEventRecord(s->ready, s->ctl));
  // Each step: a slot copies its first packet in before it waits for the new
  // dt (the copies of one step's tail and the next step's head overlap the
  // dt update); the control stream waits for every slot's last stage-2 launch
  // (not its copy-out) before it computes the next dt.  With a host share the
  // host reads dt first (it computes with it), then queues the GPU packets,
  // advances its own packets while they run, and folds its rate in.
  for (int step = 0; step < nsteps && good; ++step) {
    DevTime h;
    if (split) {
      good = ok(hipMemcpyAsync(&h, s->d_time, sizeof(DevTime), hipMemcpyDeviceToHost, s->ctl)) &&
             ok(hipStreamSynchronize(s->ctl));
    }
    std::vector<char> waited(ns, 0);
    for (int u = 0; u < nu && good; ++u) {
      const int k = s->uslot[u];
      auto &sl = s->slots[k];
      copy_in(u, sl);
      if (!waited[k]) {
        good = good && ok(hipStreamWaitEvent(sl.stream, s->ready, 0));
        waited[k] = 1;
      }
      for (int stage = 1; stage <= 2; ++stage)
        good = good && ok(hyd::launch_stage(s->ndim, is_mixed(prec), stage, s->wl[u].kmask, speeds_of(prec),
                                            recon_of(prec), eos_of(prec), s->wl[u].nitems, sl.stream,
                                            slot_args(s, sl, s->wl[u], stage, gamma)));
      if (u == lastu[k]) done(sl);
      good = good && ok(hipMemcpyAsync(s->host + s->uhost[u], sl.state, (size_t)s->ulen[u] * sizeof(double),
                                       hipMemcpyDeviceToHost, sl.stream));
    }
    // a failed earlier step leaves dt NaN: the host share then does nothing either
    if (split && good && std::fabs(h.dt) <= DBL_MAX) {
      H.dt = h.dt;
      H.stage = 1;
      H.src = s->cpu_un.data();
      H.un = nullptr;
      H.dst = s->cpu_u1p.data();
      hyd::HostRate r = hyd::host_run(H, s->cpu_threads, false);
      H.stage = 2;
      H.src = s->cpu_u1p.data();
      H.un = s->cpu_un.data();
      H.dst = s->cpu_un.data();  // Un+1 over Un: stage 2 reads Un only at the cell it writes
      r = hyd::host_run(H, s->cpu_threads, false);
      fold(r);
    }
    good = good && ok(hyd::launch_finalize(s->d_time, cfl, 0, s->ctl));
    good = good && ok(hipEventRecord(s->ready, s->ctl));
  }
  for (auto &sl : s->slots) done(sl);  // the last copies back
  DevTime h;
  if (good) good = ok(hipMemcpyAsync(&h, s->d_time, sizeof(DevTime), hipMemcpyDeviceToHost, s->ctl));
  if (good) good = ok(hipStreamSynchronize(s->ctl));
  if (!good) {
    for (auto &sl : s->slots) (void)hipStreamSynchronize(sl.stream);
    return fail(HYDRO_EDEVICE, std::string("stream run: ") + hipGetErrorString(hipGetLastError()));
  }
  if (t_out) *t_out = h.t;
  if (h.status) return nonphys(h);
  return HYDRO_OK;
}

hydro_status hydro_stream_set_cpu_share(hydro_stream *s, int32_t cpu_packets, int32_t nthreads) {
  if (!s) return fail(HYDRO_EINVAL, "stream is null");
  const int np = (int)s->pstart.size() - 1;
  if (cpu_packets < 0 || cpu_packets > np) return fail(HYDRO_EINVAL, "cpu_packets must be in 0..npackets");
  if (nthreads < 0) return fail(HYDRO_EINVAL, "nthreads must be >= 0");
  if (cpu_packets > 0 && s->prec != HYDRO_FP64 && s->prec != HYDRO_FP32_FP64)
    return fail(HYDRO_EINVAL, "the host share runs Davis bounds, primitive PLM and the gamma law only");
  const int nb = (int)s->desc.size();
  int64_t len = 0;
  for (int p = np - cpu_packets; p < np; ++p) len += s->plen[p];
  std::vector<double> u1;
  try {
    u1.resize((size_t)len);
  } catch (...) {
    return fail(HYDRO_ENOMEM, "host first-stage buffer allocation failed");
  }
  // the GPU's units first: on an error the stream keeps its previous split
  hydro_status st = build_units(s, s->unit_bytes, cpu_packets);
  if (st) return st;
  s->cpu_u1.swap(u1);
  s->cpu_un.assign(nb, nullptr);
  s->cpu_u1p.assign(nb, nullptr);
  s->cpu_ids.clear();
  int64_t base = 0;
  for (int p = np - cpu_packets; p < np; ++p) {
    for (int b = s->pstart[p]; b < s->pstart[p + 1]; ++b) {
      s->cpu_ids.push_back(b);
      s->cpu_un[b] = s->host + s->desc[b].offset;
      s->cpu_u1p[b] = s->cpu_u1.data() + base + (s->desc[b].offset - s->phost[p]);
    }
    base += s->plen[p];
  }
  s->cpu_packets = cpu_packets;
  s->cpu_threads = nthreads > 0 ? nthreads : std::max(1u, std::thread::hardware_concurrency());
  return HYDRO_OK;
}

hydro_status hydro_stream_set_unit_bytes(hydro_stream *s, int64_t min_bytes) {
  if (!s) return fail(HYDRO_EINVAL, "stream is null");
  if (min_bytes < 0) return fail(HYDRO_EINVAL, "min_bytes must be >= 0");
  return build_units(s, min_bytes, s->cpu_packets);
}

}  // extern "C"

extern "C" {

// ------------------------------------------------------------------ tuning
hydro_status hydro_batch_set_tiling(hydro_batch *b, int32_t edge, int32_t tile, int32_t zchunk) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  if (tile < 0 || tile > TILE_FUSED)
    return fail(HYDRO_EINVAL, "tile must be 0 (16x16), 1 (8x8), 2..4 (16x16 z-runs) or 5 (fused step)");
  if (zchunk < 0) return fail(HYDRO_EINVAL, "zchunk must be >= 0");
  if (tile == TILE_FUSED) {
    if (edge != 8 || zchunk != 0) return fail(HYDRO_EINVAL, "the fused step takes whole 8^3 blocks (edge 8, zchunk 0)");
    if (is_mixed(b->prec) ? b->prec != HYDRO_FP32_FP64 : b->prec != HYDRO_FP64)
      return fail(HYDRO_EINVAL, "the fused step runs Davis bounds, primitive PLM and the gamma law only");
    for (int id : b->ids)
      if (block_class(b->m->desc[id], b->m->ndim) == 8 && !fusable(b->m->desc[id], b->m->ndim))
        return fail(HYDRO_EINVAL, "the fused step needs every block of the class periodic on itself (3D, 8^3)");
  }
  if (tile != 1 && tile != TILE_FUSED && edge > 0 && edge % 16)
    return fail(HYDRO_EINVAL, "16x16 tiles need an edge multiple of 16");
  if (tile >= 2 && zchunk != 0) return fail(HYDRO_EINVAL, "z-runs take whole blocks (zchunk 0)");
  TileCfg c;
  c.tile = tile;
  c.zchunk = zchunk;
  const auto prev = b->cfg;
  b->cfg[edge] = c;
  hydro_status st = rebuild_batch_items(b);
  if (st) b->cfg = prev;  // the work list in use still follows the previous settings
  return st;
}

hydro_status hydro_batch_set_launch(hydro_batch *b, int32_t grid, int32_t xcd_remap) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  if (grid < 0) return fail(HYDRO_EINVAL, "grid must be >= 0");
  if (xcd_remap != 0 && xcd_remap != 1) return fail(HYDRO_EINVAL, "xcd_remap must be 0 or 1");
  if (grid != b->grid || xcd_remap != b->remap) {
    b->grid = grid;
    b->remap = xcd_remap;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
  }
  return HYDRO_OK;
}

hydro_status hydro_batch_set_occupancy(hydro_batch *b, int32_t waves) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  if (waves != 0 && (waves < 2 || waves > 4)) return fail(HYDRO_EINVAL, "waves must be 0 (default) or 2..4");
  if (waves != 0 && b->prec != HYDRO_FP64 && b->prec != HYDRO_FP32_FP64)
    return fail(HYDRO_EINVAL, "an occupancy request applies to the default method only");
  if (waves != b->occ) {
    b->occ = waves;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
  }
  return HYDRO_OK;
}

hydro_status hydro_batch_get_config(hydro_batch *b, int32_t *out, int32_t nclass_max, int32_t *nclass) {
  if (!b || !out || !nclass || nclass_max < 0) return fail(HYDRO_EINVAL, "bad arguments");
  std::map<int, int64_t> cells, tiles;
  for (int id : b->ids) {
    const hydro_block_desc &d = b->m->desc[id];
    cells[block_class(d, b->m->ndim)] += (int64_t)d.n[0] * d.n[1] * d.n[2];
    tiles[block_class(d, b->m->ndim)] += (int64_t)(d.n[0] / 16) * (d.n[1] / 16);
  }
  out[0] = b->grid;
  out[1] = b->remap;
  out[2] = b->occ;
  int k = 0;
  for (auto &kv : cells) {
    if (k < nclass_max) {
      TileCfg c;
      auto f = b->cfg.find(kv.first);
      if (f != b->cfg.end()) c = f->second;
      const hydro_block_desc *any = nullptr;
      for (int id : b->ids)
        if (block_class(b->m->desc[id], b->m->ndim) == kv.first) {
          any = &b->m->desc[id];
          break;
        }
      const bool can16 = any && any->n[0] % 16 == 0 && any->n[1] % 16 == 0;
      out[3 + 4 * k + 0] = kv.first;
      // the tiling in effect: 8x8, 16x16, the z-run length, or the fused step
      int tile = 1;
      if (c.tile == TILE_FUSED) {
        tile = TILE_FUSED;
      } else if (can16 && c.tile != 1) {
        const bool whole = b->m->ndim == 3 && (c.zchunk == 0 || (any && c.zchunk >= any->n[2]));
        // runs chain blocks along their +z links: a class without them runs single blocks
        const bool zlinked = any && any->face_kind[5] == HYDRO_NBR;
        const int run = !whole || !zlinked ? 1 : (c.tile < 0 ? default_run(b->m, tiles[kv.first]) : std::max(c.tile, 1));
        tile = run > 1 ? run : 0;
      }
      out[3 + 4 * k + 1] = tile;
      out[3 + 4 * k + 2] = c.zchunk;
      out[3 + 4 * k + 3] = (int32_t)(kv.second & 0x7fffffff);
    }
    ++k;
  }
  *nclass = k;
  return HYDRO_OK;
}

// Device time (ms) of one RK step of work list wl: the median over `reps`
// launches of each stage, summed.  Stage 1 reads the state and writes the U1
// scratch, as in a step.  Stage 2 takes its stencil from the state and its
// pointwise Un from the U1 scratch, and writes the U1 scratch (each thread
// reads Un only at its own cells before it writes them), so it moves the
// bytes of a real stage 2 -- a stencil source and a separate pointwise
// buffer -- while the caller's state is never modified.  Both stages are
// timed because a tiling can shift work between them (stage 2 carries Un
// and the CFL rate).
static hydro_status time_step(hydro_batch *b, const WorkList &wl, int grid, int remap, double gamma, int reps,
                              double &ms, int occ = 0) {
  hydro_mesh *m = b->m;
  const int prec = b->prec;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(HYDRO_EDEVICE, "tuning: event creation failed");
  }
  hydro_status st = HYDRO_OK;
  const double dt = 1e-30;  // the results are scratch; any positive dt
  StageArgs args[2] = {stage_args(m, wl, 1, dt, nullptr, b->d_time, gamma, 0, remap),
                       stage_args(m, wl, 2, dt, nullptr, b->d_time, gamma, 0, remap)};
  args[1].src = m->arena;
  args[1].un = m->u1;
  args[1].dst = m->u1;
  ms = 0.0;
  for (int stage = 1; stage <= 2 && !st; ++stage) {
    const StageArgs &a = args[stage - 1];
    std::vector<double> t;
    st = launch_stage_wl(m, prec, stage, wl, grid, m->stream, a, occ);  // warm-up
    for (int r = 0; r < reps && !st; ++r) {
      (void)hipEventRecord(e0, m->stream);
      st = launch_stage_wl(m, prec, stage, wl, grid, m->stream, a, occ);
      (void)hipEventRecord(e1, m->stream);
      if (!st && hipEventSynchronize(e1) != hipSuccess) st = fail(HYDRO_EDEVICE, "tuning: event sync failed");
      float f = 0;
      (void)hipEventElapsedTime(&f, e0, e1);
      t.push_back(f);
    }
    if (!st) {
      std::sort(t.begin(), t.end());
      ms += t[t.size() / 2];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Results of the listed blocks after one launch of the given stage with
// tiling `cfg`, written to the U1 scratch and read back: stage 1 from the
// state; stage 2 with the state as both its stencil source and its pointwise
// Un (a valid stage-2 input whose every neighbour value is defined, so the
// stage-2 code path -- z-run marching, the Un stream, the rate epilogue -- is
// compared on the sample alone).
static hydro_status stage_sample(hydro_batch *b, int stage, const std::vector<int32_t> &ids,
                                 const std::map<int, TileCfg> &cfg, double gamma, std::vector<double> &out,
                                 int occ = 0) {
  hydro_mesh *m = b->m;
  std::vector<WorkItem> items;
  int kmask;
  WorkList wl;
  build_items(m, ids, cfg, items, kmask);
  hydro_status st = upload_items(items, kmask, wl, m->stream);
  if (st) return st;
  StageArgs a = stage_args(m, wl, stage, 1e-3, nullptr, b->d_time, gamma, 0);
  a.src = m->arena;
  a.un = m->arena;
  a.dst = m->u1;
  st = launch_stage_wl(m, b->prec, stage, wl, 0, m->stream, a, occ);
  out.clear();
  for (int id : ids) {
    if (st) break;
    const hydro_block_desc &d = m->desc[id];
    const size_t len = (size_t)5 * d.n[0] * d.n[1] * d.n[2];
    const size_t o = out.size();
    out.resize(o + len);
    if (hipMemcpyAsync(out.data() + o, m->u1 + d.offset, len * sizeof(double), hipMemcpyDeviceToHost, m->stream) !=
        hipSuccess)
      st = fail(HYDRO_EDEVICE, "tuning: readback failed");
  }
  if (!st && hipStreamSynchronize(m->stream) != hipSuccess) st = fail(HYDRO_EDEVICE, "tuning: sync failed");
  (void)hipFree(wl.d_items);
  return st;
}

// Device buffer freed on scope exit (tuning temporaries).
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes > 0 ? bytes : 1); }
};

// One SSP-RK2 step (dt 1e-3) of the listed self-periodic blocks, copied into
// a compact temporary arena: with the two stage kernels of the default tiling
// (fused = false) or with the fused kernel.  `out` receives the result in the
// compact layout.  The caller's arena and the mesh's scratch are not written.
static hydro_status fused_sample_step(hydro_batch *b, const std::vector<int32_t> &ids, bool fused, double gamma,
                                      std::vector<double> &out) {
  hydro_mesh *m = b->m;
  const int n = (int)ids.size();
  std::vector<hydro_block_desc> local(n);
  int64_t len = 0;
  for (int i = 0; i < n; ++i) {
    local[i] = m->desc[ids[i]];
    local[i].offset = len;
    len += 5 * (int64_t)local[i].n[0] * local[i].n[1] * local[i].n[2];
  }
  std::vector<DevBlock> hb(n);
  for (int i = 0; i < n; ++i) hb[i] = make_devblock(local.data(), i, m->ndim);
  hydro_mesh view;
  view.ndim = m->ndim;
  view.nblocks = n;
  view.desc = local;
  view.num_cu = m->num_cu;
  std::vector<int32_t> lid(n);
  for (int i = 0; i < n; ++i) lid[i] = i;
  std::vector<WorkItem> items;
  int kmask = 0;
  build_items(&view, lid, {}, items, kmask);
  DevBuf state, u1, blocks, its, dids, tm;
  if (state.alloc(len * sizeof(double)) || u1.alloc(len * sizeof(double)) || blocks.alloc(n * sizeof(DevBlock)) ||
      its.alloc(items.size() * sizeof(WorkItem)) || dids.alloc(n * sizeof(int32_t)) || tm.alloc(sizeof(DevTime)))
    return fail(HYDRO_ENOMEM, "tuning: hipMalloc of the fused-step sample failed");
  hipStream_t s = m->stream;
  HIP_TRY(hipMemcpyAsync(blocks.p, hb.data(), n * sizeof(DevBlock), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(its.p, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dids.p, lid.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIP_TRY(hyd::launch_reset(static_cast<DevTime *>(tm.p), s));
  double *st = static_cast<double *>(state.p);
  for (int i = 0; i < n; ++i)
    HIP_TRY(hipMemcpyAsync(st + local[i].offset, m->arena + m->desc[ids[i]].offset,
                           5 * (size_t)local[i].n[0] * local[i].n[1] * local[i].n[2] * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  const double dt = 1e-3;
  const bool mixed = is_mixed(b->prec);
  if (fused) {
    hyd::FusedArgs a;
    a.blocks = static_cast<DevBlock *>(blocks.p);
    a.ids = static_cast<int32_t *>(dids.p);
    a.nblocks = n;
    a.rate_only = 0;
    a.xcd_remap = 1;
    a.state = st;
    a.dt = dt;
    a.dt_dev = nullptr;
    a.acc = static_cast<DevTime *>(tm.p);
    a.gamma = gamma;
    HIP_TRY(hyd::launch_fused(mixed, n, s, a));
  } else {
    StageArgs a;
    a.blocks = static_cast<DevBlock *>(blocks.p);
    a.items = static_cast<WorkItem *>(its.p);
    a.nitems = (int)items.size();
    a.reset_time = 1;
    a.xcd_remap = 1;
    a.src = st;
    a.un = st;
    a.dst = static_cast<double *>(u1.p);
    a.dt = dt;
    a.dt_dev = nullptr;
    a.acc = static_cast<DevTime *>(tm.p);
    a.gamma = gamma;
    HIP_TRY(hyd::launch_stage(m->ndim, mixed, 1, kmask, 0, 0, 0, a.nitems, s, a));
    a.reset_time = 0;
    a.src = static_cast<double *>(u1.p);
    a.dst = st;
    HIP_TRY(hyd::launch_stage(m->ndim, mixed, 2, kmask, 0, 0, 0, a.nitems, s, a));
  }
  out.resize(len);
  HIP_TRY(hipMemcpyAsync(out.data(), st, len * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HYDRO_OK;
}

// Median device time (ms) of `reps` whole steps of the batch as configured:
// the stage-1 and stage-2 launches over its work list and the fused launch
// of its fused classes, on a copy of the state in the mesh's scratch buffer
// (stage 1 from the arena into the scratch; stage 2 with the arena as
// stencil and the scratch as Un and output; the fused step in place in the
// scratch), so the caller's arena is not written.
static hydro_status time_full(hydro_batch *b, double gamma, int reps, double &ms) {
  hydro_mesh *m = b->m;
  const int prec = b->prec;
  HIP_TRY(hipMemcpyAsync(m->u1, m->arena, (size_t)m->arena_len * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  const double dt = 1e-30;
  StageArgs a1 = stage_args(m, b->wl, 1, dt, nullptr, b->d_time, gamma, 0, b->remap);
  StageArgs a2 = stage_args(m, b->wl, 2, dt, nullptr, b->d_time, gamma, 0, b->remap);
  a2.src = m->arena;
  a2.un = m->u1;
  a2.dst = m->u1;
  const hyd::FusedArgs af = fused_args(m, b->d_fused, b->nfused, m->u1, dt, nullptr, b->d_time, gamma, 0, b->remap);
  auto step = [&]() -> hydro_status {  // as in a captured step: the fused launch beside the stage launches
    hydro_status s2 = HYDRO_OK;
    if (b->nfused > 0 &&
        (hipEventRecord(b->fork_ev, m->stream) != hipSuccess ||
         hipStreamWaitEvent(b->side_stream, b->fork_ev, 0) != hipSuccess ||
         hyd::launch_fused(is_mixed(prec), fused_grid(b), b->side_stream, af) != hipSuccess ||
         hipEventRecord(b->join_ev, b->side_stream) != hipSuccess))
      s2 = fail(HYDRO_EDEVICE, "tuning: fused launch failed");
    if (!s2) s2 = launch_stage_wl(m, prec, 1, b->wl, b->grid, m->stream, a1, b->occ);
    if (!s2) s2 = launch_stage_wl(m, prec, 2, b->wl, b->grid, m->stream, a2, b->occ);
    if (!s2 && b->nfused > 0 && hipStreamWaitEvent(m->stream, b->join_ev, 0) != hipSuccess)
      s2 = fail(HYDRO_EDEVICE, "tuning: fused join failed");
    return s2;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(HYDRO_EDEVICE, "tuning: event creation failed");
  }
  hydro_status st = step();  // warm-up
  std::vector<double> t;
  for (int r = 0; r < reps && !st; ++r) {
    (void)hipEventRecord(e0, m->stream);
    st = step();
    (void)hipEventRecord(e1, m->stream);
    if (!st && hipEventSynchronize(e1) != hipSuccess) st = fail(HYDRO_EDEVICE, "tuning: event sync failed");
    float f = 0;
    (void)hipEventElapsedTime(&f, e0, e1);
    t.push_back(f);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  std::sort(t.begin(), t.end());
  ms = t[t.size() / 2];
  return HYDRO_OK;
}

static hydro_status autotune(hydro_batch *b, double gamma, int32_t reps);

hydro_status hydro_batch_autotune(hydro_batch *b, double gamma, int32_t reps) {
  if (!b) return fail(HYDRO_EINVAL, "batch is null");
  if (reps < 1) return fail(HYDRO_EINVAL, "reps must be >= 1");
  if (!std::isfinite(gamma) || gamma <= 1.0) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  const auto cfg = b->cfg;
  const int grid = b->grid, remap = b->remap, occ = b->occ;
  hydro_status st = autotune(b, gamma, reps);
  if (st) {  // back to the settings the batch had (its message kept)
    const std::string msg = g_err;
    b->cfg = cfg;
    (void)rebuild_batch_items(b);
    (void)hydro_batch_set_launch(b, grid, remap);
    (void)hydro_batch_set_occupancy(b, occ);
    std::snprintf(g_err, sizeof(g_err), "%s", msg.c_str());
  }
  return st;
}

static hydro_status autotune(hydro_batch *b, double gamma, int32_t reps) {
  hydro_mesh *m = b->m;
  const double tol = is_mixed(b->prec) ? 1e-6 : 1e-13;
  std::vector<int> fused_ok;  // classes whose fused step passed the parity check
  std::map<int, std::vector<int32_t>> cls;
  for (int id : b->ids) cls[block_class(m->desc[id], m->ndim)].push_back(id);
  for (auto &kv : cls) {
    const int edge = kv.first;
    const std::vector<int32_t> &ids = kv.second;
    const hydro_block_desc &d0 = m->desc[ids[0]];
    bool can16 = true;
    for (int id : ids) can16 = can16 && m->desc[id].n[0] % 16 == 0 && m->desc[id].n[1] % 16 == 0;
    std::vector<TileCfg> cands;
    std::vector<int> zcs = {0};
    if (m->ndim == 3)
      for (int zc : {d0.n[2] / 2, d0.n[2] / 4})
        if (zc >= 4) zcs.push_back(zc);
    for (int tile : {0, 1}) {
      if (tile == 0 && !can16) continue;
      for (int zc : zcs) {
        TileCfg c;
        c.tile = tile;
        c.zchunk = zc;
        cands.push_back(c);
      }
    }
    bool zlinked = true;  // z-runs chain blocks along their +z links
    for (int id : ids) zlinked = zlinked && m->desc[id].face_kind[5] == HYDRO_NBR;
    if (can16 && m->ndim == 3 && zlinked)
      for (int k : {2, 4}) {
        TileCfg c;
        c.tile = k;
        cands.push_back(c);
      }
    // parity reference: default tiling on a sample of blocks, both stages
    std::vector<int32_t> sample(ids.begin(), ids.begin() + std::min<size_t>(ids.size(), 64));
    std::vector<double> ref[2], got;
    hydro_status st = HYDRO_OK;
    for (int stage = 1; stage <= 2 && !st; ++stage) st = stage_sample(b, stage, sample, {}, gamma, ref[stage - 1]);
    if (st) return st;
    double best = 1e300;
    TileCfg bestc;
    for (const TileCfg &c : cands) {
      std::map<int, TileCfg> one;
      one[edge] = c;
      bool ok = true;
      for (int stage = 1; stage <= 2 && ok; ++stage) {
        st = stage_sample(b, stage, sample, one, gamma, got);
        if (st) return st;
        const std::vector<double> &r = ref[stage - 1];
        ok = got.size() == r.size();
        double scale = 0.0;
        for (double x : r) scale = std::max(scale, std::fabs(x));
        for (size_t i = 0; ok && i < r.size(); ++i)
          ok = std::fabs(got[i] - r[i]) <= tol * (std::fabs(r[i]) + 1e-6 * scale);
      }
      if (!ok) continue;
      std::vector<WorkItem> items;
      int kmask;
      WorkList wl;
      build_items(m, ids, one, items, kmask);
      st = upload_items(items, kmask, wl, m->stream);
      if (st) return st;
      double ms = 0;
      st = time_step(b, wl, 0, b->remap, gamma, reps, ms);
      (void)hipFree(wl.d_items);
      if (st) return st;
      if (ms < best) {
        best = ms;
        bestc = c;
      }
    }
    // the fused step of self-periodic 8^3 blocks: both stages in one launch,
    // kept when it passes the same parity check (one full step on the sample
    // against the default two-launch step) and beats the best tiling's two
    // stage launches
    bool all_fusable = edge == 8 && (b->prec == HYDRO_FP64 || b->prec == HYDRO_FP32_FP64);
    for (int id : ids) all_fusable = all_fusable && fusable(m->desc[id], m->ndim);
    if (all_fusable) {
      std::vector<double> r2, g2;
      st = fused_sample_step(b, sample, false, gamma, r2);
      if (!st) st = fused_sample_step(b, sample, true, gamma, g2);
      if (st) return st;
      bool ok = r2.size() == g2.size();
      double scale = 0.0;
      for (double x : r2) scale = std::max(scale, std::fabs(x));
      for (size_t i = 0; ok && i < r2.size(); ++i) ok = std::fabs(g2[i] - r2[i]) <= tol * (std::fabs(r2[i]) + 1e-6 * scale);
      if (ok) fused_ok.push_back(edge);  // decided on the whole step below
    }
    b->cfg[edge] = bestc;
  }
  hydro_status st = rebuild_batch_items(b);
  if (st) return st;
  // launch: one workgroup per item or persistent grids of k workgroups per CU,
  // each with and without the XCD renumbering
  double best = 1e300;
  int bestg = 0, bestr = 1;
  for (int r : {1, 0})
    for (int g : {0, 2 * m->num_cu, 4 * m->num_cu, 8 * m->num_cu}) {
      if (g > 0 && g >= b->wl.nitems) continue;
      double ms = 0;
      st = time_step(b, b->wl, g, r, gamma, reps, ms);
      if (st) return st;
      if (ms < best) {
        best = ms;
        bestg = g;
        bestr = r;
      }
    }
  st = hydro_batch_set_launch(b, bestg, bestr);
  if (st) return st;
  // the fused step of a class, kept when the whole step (stage launches of
  // the other classes plus the fused launch) is faster with it: the class's
  // share of the stage launches and the separate launch interact, so the
  // class's own times do not decide it
  for (int edge : fused_ok) {
    const TileCfg keep = b->cfg[edge];
    double t_keep = 0, t_fused = 0;
    st = time_full(b, gamma, reps, t_keep);
    if (st) return st;
    TileCfg f;
    f.tile = TILE_FUSED;
    b->cfg[edge] = f;
    st = rebuild_batch_items(b);
    if (!st) st = time_full(b, gamma, reps, t_fused);
    if (st) return st;
    if (!(t_fused < t_keep)) {
      b->cfg[edge] = keep;
      st = rebuild_batch_items(b);
      if (st) return st;
    }
  }
  // occupancy: the register budget of 2, 3 or 4 waves per SIMD against the
  // kernels' own (default method only), each parity-checked on the sample of
  // every class against the default budget
  int besto = 0;
  if (b->prec == HYDRO_FP64 || b->prec == HYDRO_FP32_FP64) {
    // the baseline again: a class moved to the fused step has left the work
    // list since the launch shapes were timed
    st = time_step(b, b->wl, bestg, bestr, gamma, reps, best);
    if (st) return st;
    std::vector<int32_t> sample;
    for (auto &kv : cls)
      sample.insert(sample.end(), kv.second.begin(), kv.second.begin() + std::min<size_t>(kv.second.size(), 16));
    std::vector<double> ref[2], got;
    for (int stage = 1; stage <= 2 && !st; ++stage) st = stage_sample(b, stage, sample, b->cfg, gamma, ref[stage - 1]);
    if (st) return st;
    for (int o : {2, 3, 4}) {
      bool ok = true;
      for (int stage = 1; stage <= 2 && ok; ++stage) {
        st = stage_sample(b, stage, sample, b->cfg, gamma, got, o);
        if (st) return st;
        const std::vector<double> &rr = ref[stage - 1];
        ok = got.size() == rr.size();
        double scale = 0.0;
        for (double x : rr) scale = std::max(scale, std::fabs(x));
        for (size_t i = 0; ok && i < rr.size(); ++i)
          ok = std::fabs(got[i] - rr[i]) <= tol * (std::fabs(rr[i]) + 1e-6 * scale);
      }
      if (!ok) continue;
      double ms = 0;
      st = time_step(b, b->wl, bestg, bestr, gamma, reps, ms, o);
      if (st) return st;
      if (ms < best) {
        best = ms;
        besto = o;
      }
    }
  }
  return hydro_batch_set_occupancy(b, besto);
}

}  // extern "C"

// ------------------------------------------------------- allocation-free step
namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;  // per GPU
constexpr int kStaticMaxBlocks = 4096;
constexpr int kSetupChunk = 16;  // blocks per setup launch (kernel arguments <= 4 KiB)
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Tiling of a block in the allocation-free step: 16x16 tiles where both
// extents allow, else 8x8 tiles packed four to a work item within the block.
int static_items_of(const hydro_block_desc &d, bool *t16) {
  *t16 = (d.n[0] % 16 == 0) && (d.n[1] % 16 == 0);
  const int T = *t16 ? 16 : 8;
  const int tiles = (d.n[0] / T) * (d.n[1] / T);
  return *t16 ? tiles : (tiles + 3) / 4;
}

// Up to kSetupChunk blocks' resolved table entries, passed to the setup
// kernel by value, so that the host keeps no buffer alive after the launch.
struct SetupChunk {
  DevBlock blk[kSetupChunk];
  int32_t id[kSetupChunk];     // block id of entry g
  int32_t item0[kSetupChunk];  // first work item of block id[g]
  int32_t count;
};
static_assert(sizeof(SetupChunk) <= 4096, "setup kernel arguments must stay within 4 KiB");
static_assert(sizeof(DevBlock) == 176 && sizeof(WorkItem) == 40, "the static step's size limit in hydro.h counts these sizes");

std::atomic<void *> g_scratch_addr[kMaxDevices];
std::pair<int64_t, int64_t> g_static_ranges[kStaticMaxBlocks];
std::mutex g_static_ranges_mu;

}  // namespace

// The fixed device scratch of hydro_step_static: the time record, the block
// table, the work list and the first-stage state of one call.  Each GPU holds
// its own copy from the library's first use there until the process ends.
// Host code never passes this name to a kernel: it uses the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// One workgroup per block of the chunk: the table entry, then the block's
// work items (one per 16x16 tile, or one per four 8x8 tiles of the block with
// empty slots marked -1), whole z range.
__global__ void k_static_setup(SetupChunk c, DevBlock *table, WorkItem *items) {
  const int g = blockIdx.x;
  if (g >= c.count) return;
  const DevBlock &B = c.blk[g];
  const int id = c.id[g];
  if (threadIdx.x == 0) table[id] = B;
  const bool t16 = (B.n[0] % 16 == 0) && (B.n[1] % 16 == 0);
  const int T = t16 ? 16 : 8;
  const int tx = B.n[0] / T, ntile = tx * (B.n[1] / T);
  const int nitem = t16 ? ntile : (ntile + 3) / 4;
  for (int j = threadIdx.x; j < nitem; j += blockDim.x) {
    WorkItem it;
    it.kind = t16 ? hyd::KIND_T16 : hyd::KIND_T8;
    it.z0 = 0;
    it.z1 = (int16_t)B.n[2];
    for (int s = 0; s < 4; ++s) {
      const int t = t16 ? (s == 0 ? j : -1) : 4 * j + s;
      const bool on = t >= 0 && t < ntile;
      it.block[s] = on ? id : -1;
      it.x0[s] = (int16_t)(on ? (t % tx) * T : 0);
      it.y0[s] = (int16_t)(on ? (t / tx) * T : 0);
    }
    items[c.item0[g] + j] = it;
  }
}

#define HIP_TRYF(call)                                                                                \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return failf(HYDRO_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));         \
  } while (0)

extern "C" {

hydro_status hydro_step_static(const hydro_block_desc *blocks, int32_t nblocks, int32_t ndim, double *arena,
                               int64_t arena_len, int32_t precision, double dt, double gamma, void *stream) {
  if (nblocks > kStaticMaxBlocks)
    return failf(HYDRO_EINVAL, "static step: %d blocks, at most %d", (int)nblocks, kStaticMaxBlocks);
  hydro_status st;
  {  // the overlap check sorts block ranges in a fixed host array (no
     // allocation, and nothing large on the caller's stack)
    std::lock_guard<std::mutex> lock(g_static_ranges_mu);
    st = validate_blocks(blocks, nblocks, ndim, arena, arena_len, g_static_ranges);
  }
  if (st) return st;
  if (!prec_valid(precision)) return failf(HYDRO_EINVAL, "static step: bad precision");
  if (!finite_pos(dt)) return failf(HYDRO_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(gamma) || gamma <= 1.0) return failf(HYDRO_EINVAL, "gamma must be finite and > 1");
  // scratch layout: time record | block table | work list | first-stage state
  int64_t nitems = 0;
  int kmask = 0;
  for (int b = 0; b < nblocks; ++b) {
    bool t16 = false;
    nitems += static_items_of(blocks[b], &t16);
    kmask |= t16 ? 1 : 2;
  }
  const size_t off_blocks = align_up(sizeof(DevTime));
  const size_t off_items = off_blocks + align_up((size_t)nblocks * sizeof(DevBlock));
  const size_t off_u1 = off_items + align_up((size_t)nitems * sizeof(WorkItem));
  const size_t need = off_u1 + (size_t)arena_len * sizeof(double);
  if (need > kStaticScratchBytes || nitems > INT_MAX)
    return failf(HYDRO_EINVAL,
                 "static step: the mesh needs %zu bytes of scratch (first-stage state of arena_len doubles plus "
                 "tables); the static scratch holds %zu",
                 need, kStaticScratchBytes);
  int dev = 0;
  HIP_TRYF(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return failf(HYDRO_EDEVICE, "static step: device %d out of range", dev);
  void *base = g_scratch_addr[dev].load(std::memory_order_acquire);
  if (!base) {  // first call on this device: look up this GPU's copy of the array
    void *p = nullptr;
    HIP_TRYF(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return failf(HYDRO_EDEVICE, "static step: no device address for the scratch array");
    g_scratch_addr[dev].store(p, std::memory_order_release);
    base = p;
  }
  unsigned char *sb = static_cast<unsigned char *>(base);
  DevTime *d_time = reinterpret_cast<DevTime *>(sb);
  DevBlock *d_blocks = reinterpret_cast<DevBlock *>(sb + off_blocks);
  WorkItem *d_items = reinterpret_cast<WorkItem *>(sb + off_items);
  double *d_u1 = reinterpret_cast<double *>(sb + off_u1);
  hipStream_t s = (hipStream_t)stream;

  SetupChunk chunk;
  int32_t item0 = 0;
  for (int b0 = 0; b0 < nblocks; b0 += kSetupChunk) {
    std::memset(&chunk, 0, sizeof(chunk));
    chunk.count = std::min(kSetupChunk, nblocks - b0);
    for (int g = 0; g < chunk.count; ++g) {
      const int b = b0 + g;
      bool t16 = false;
      chunk.blk[g] = make_devblock(blocks, b, ndim);
      chunk.id[g] = b;
      chunk.item0[g] = item0;
      item0 += static_items_of(blocks[b], &t16);
    }
    hipLaunchKernelGGL(k_static_setup, dim3(chunk.count), dim3(256), 0, s, chunk, d_blocks, d_items);
    HIP_TRYF(hipGetLastError());
  }
  StageArgs a;
  a.blocks = d_blocks;
  a.items = d_items;
  a.nitems = (int32_t)nitems;
  a.reset_time = 1;  // stage 1 clears the time record's accumulators
  a.xcd_remap = 1;
  a.src = arena;
  a.un = arena;
  a.dst = d_u1;
  a.dt = dt;
  a.dt_dev = nullptr;
  a.acc = d_time;
  a.gamma = gamma;
  const bool mixed = is_mixed(precision);
  HIP_TRYF(hyd::launch_stage(ndim, mixed, 1, kmask, speeds_of(precision), recon_of(precision), eos_of(precision),
                             (int)nitems, s, a));
  a.reset_time = 0;
  a.src = d_u1;
  a.dst = arena;
  HIP_TRYF(hyd::launch_stage(ndim, mixed, 2, kmask, speeds_of(precision), recon_of(precision), eos_of(precision),
                             (int)nitems, s, a));
  return HYDRO_OK;
}

}  // extern "C"
