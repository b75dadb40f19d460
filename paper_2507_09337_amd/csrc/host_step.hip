// host_step.hip -- the host-core kernel of the CPU/GPU split of host-resident
// packets: one SSP-RK2 stage (or the CFL rate) of a set of blocks computed by
// host threads, in place in host memory, while the GPU advances the other
// packets.
//
// Arithmetic: the FP64 point functions of the GPU's FP64 tile (recovery,
// minmod PLM, HLLC with Davis bounds, CFL rate; stage_kernels.h, compiled
// here for the host with contraction off), the same face frames and the same
// update order, so a block advanced here equals, bit for bit, the same block
// advanced by the FP64 stage kernels.  Per block and stage: the stage
// source's primitives on the block padded by two guard layers (face slabs
// only: the face-based stencil never reads edge or corner guards), gathered
// by the guard rules of the block's faces; the x, y and z face fluxes; the
// update dU = sum_d (dt/dx_d)(F_lo - F_hi) in x, y, z order.
//
// Threads take blocks from a shared counter; each keeps its own scratch and
// its own rate maximum and non-physical flag, merged at the end.
#include <algorithm>
#include <atomic>
#include <climits>
#include <thread>
#include <vector>

#include "host_step.h"
#include "stage_kernels.h"

namespace hyd {
namespace {

struct Scratch {
  std::vector<double> W;   // [5][pz][py][px] primitives with the guard slabs
  std::vector<double> F;   // fluxes of one direction, [5][faces]
  std::vector<double> dU;  // [5][ncell] stage increment
};

// Source of coordinate c (possibly outside [0, n)) along one axis of block b
// for face f = 2 * axis + (c >= n): the block whose data it is and the
// coordinate inside that block.
inline void guard_source(const hydro_block_desc *desc, int b, int axis, int c, int &blk, int &cc) {
  const hydro_block_desc &d = desc[b];
  const int n = d.n[axis];
  blk = b;
  cc = c;
  if (c >= 0 && c < n) return;
  const int f = 2 * axis + (c >= n ? 1 : 0);
  switch (d.face_kind[f]) {
    case HYDRO_OUTFLOW:
      cc = c < 0 ? 0 : n - 1;
      break;
    case HYDRO_PERIODIC_SELF:
      cc = c < 0 ? n + c : c - n;
      break;
    default:  // HYDRO_NBR: the far layers of the neighbour (same tangential extents)
      blk = d.nbr[f];
      cc = c < 0 ? desc[blk].n[axis] + c : c - n;
      break;
  }
}

void block_stage(const HostStage &H, int b, Scratch &S, HostRate &r) {
#pragma clang fp contract(off)
  const hydro_block_desc &d = H.desc[b];
  const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
  const bool three = H.ndim == 3;
  const int g = 2, px = nx + 2 * g, py = ny + 2 * g, pz = three ? nz + 2 * g : 1, zo = three ? g : 0;
  const int64_t pp = (int64_t)px * py * pz, ncell = (int64_t)nx * ny * nz;
  const double gamma = H.gamma, gm1 = gamma - 1.0;
  S.W.assign(NVAR * pp, 0.0);
  auto widx = [&](int i, int j, int k) { return ((int64_t)(k + zo) * py + (j + g)) * px + (i + g); };
  // primitives of cell (i, j, k) of this block's padded view, at most one
  // coordinate outside the block
  auto gather = [&](int i, int j, int k, bool own) {
    int blk = b, ii = i, jj = j, kk = k;
    if (i < 0 || i >= nx)
      guard_source(H.desc, b, 0, i, blk, ii);
    else if (j < 0 || j >= ny)
      guard_source(H.desc, b, 1, j, blk, jj);
    else if (three && (k < 0 || k >= nz))
      guard_source(H.desc, b, 2, k, blk, kk);
    const hydro_block_desc &s = H.desc[blk];
    const int64_t vs = (int64_t)s.n[0] * s.n[1] * s.n[2];
    const double *p = H.src[blk] + ((int64_t)kk * s.n[1] + jj) * s.n[0] + ii;
    double Wd[5];
    if (!recover(p[0], p[vs], p[2 * vs], p[3 * vs], p[4 * vs], gm1, Wd) && H.stage == 2) {
      r.bad = 1;  // (stage 1 reports nothing: a bad Un was reported by the rate that gave dt)
      if (own) r.bad_block = std::min(r.bad_block, b);
    }
    const int64_t w = widx(i, j, k);
    for (int v = 0; v < NVAR; ++v) S.W[v * pp + w] = Wd[v];
  };
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) gather(i, j, k, true);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i : {-2, -1, nx, nx + 1}) gather(i, j, k, false);
  for (int k = 0; k < nz; ++k)
    for (int j : {-2, -1, ny, ny + 1})
      for (int i = 0; i < nx; ++i) gather(i, j, k, false);
  if (three)
    for (int k : {-2, -1, nz, nz + 1})
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) gather(i, j, k, false);

  const double dtd[3] = {H.dt / d.dx[0], H.dt / d.dx[1], three ? H.dt / d.dx[2] : 0.0};
  S.dU.assign(NVAR * ncell, 0.0);
  const int ndir = three ? 3 : 2;
  for (int dir = 0; dir < ndir; ++dir) {
    // faces along dir: face q lies between cells q-1 and q (q = 0 .. n_dir)
    const int fx = nx + (dir == 0), fy = ny + (dir == 1), fz = nz + (dir == 2);
    const int64_t nf = (int64_t)fx * fy * fz;
    S.F.resize(NVAR * nf);
    const int64_t step = dir == 0 ? 1 : dir == 1 ? px : (int64_t)px * py;
    const int n = dir == 0 ? 1 : dir == 1 ? 2 : 3, t1 = dir == 1 ? 1 : 2, t2 = dir == 2 ? 1 : 3;
    for (int k = 0; k < fz; ++k)
      for (int j = 0; j < fy; ++j)
        for (int i = 0; i < fx; ++i) {
          // the four cells along dir: q-2, q-1, q, q+1
          const int64_t c2 = widx(i, j, k), c0 = c2 - 2 * step;
          double wl[5], wr[5];
          for (int v = 0; v < NVAR; ++v) {
            const double *w = S.W.data() + v * pp + c0;
            plm(w[0], w[step], w[2 * step], w[3 * step], wl[v], wr[v]);
          }
          const double L[5] = {wl[0], wl[n], wl[t1], wl[t2], wl[4]};
          const double R[5] = {wr[0], wr[n], wr[t1], wr[t2], wr[4]};
          double Fr[5];
          hllc_fp64<SPEEDS_DAVIS, EOS_IDEAL>(L, R, gamma, Fr);
          double Fo[5];
          Fo[0] = Fr[0];
          Fo[n] = Fr[1];
          Fo[t1] = Fr[2];
          Fo[t2] = Fr[3];
          Fo[4] = Fr[4];
          const int64_t q = ((int64_t)k * fy + j) * fx + i;
          for (int v = 0; v < NVAR; ++v) S.F[v * nf + q] = Fo[v];
        }
    const int64_t hi = dir == 0 ? 1 : dir == 1 ? fx : (int64_t)fx * fy;
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const int64_t c = ((int64_t)k * ny + j) * nx + i, q = ((int64_t)k * fy + j) * fx + i;
          for (int v = 0; v < NVAR; ++v) {
            const double df = S.F[v * nf + q] - S.F[v * nf + q + hi];
            if (dir == 0)
              S.dU[v * ncell + c] = dtd[0] * df;
            else
              S.dU[v * ncell + c] += dtd[dir] * df;
          }
        }
  }
  // stage 1: U1 = Un + dU;  stage 2: Un+1 = Un/2 + (U1 + dU)/2, then the CFL rate of the new state
  const double *us = H.src[b];
  const double *un = H.un ? H.un[b] : nullptr;
  double *dst = H.dst[b];
  for (int64_t c = 0; c < ncell; ++c) {
    double Unew[5];
    for (int v = 0; v < NVAR; ++v) {
      const double dU = S.dU[v * ncell + c];
      Unew[v] = H.stage == 1 ? us[v * ncell + c] + dU : 0.5 * un[v * ncell + c] + 0.5 * (us[v * ncell + c] + dU);
    }
    for (int v = 0; v < NVAR; ++v) dst[v * ncell + c] = Unew[v];
    if (H.stage == 2) {
      double Wd[5];
      if (!recover(Unew[0], Unew[1], Unew[2], Unew[3], Unew[4], gm1, Wd)) {
        r.bad = 1;
        r.bad_block = std::min(r.bad_block, b);
      } else {
        r.lam = std::max(r.lam, three ? cell_rate<3>(Wd, gamma, d.dx[0], d.dx[1], d.dx[2])
                                      : cell_rate<2>(Wd, gamma, d.dx[0], d.dx[1], d.dx[2]));
      }
    }
  }
}

void block_rate(const HostStage &H, int b, HostRate &r) {
#pragma clang fp contract(off)
  const hydro_block_desc &d = H.desc[b];
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  const double *p = H.src[b];
  for (int64_t c = 0; c < ncell; ++c) {
    double Wd[5];
    if (!recover(p[c], p[ncell + c], p[2 * ncell + c], p[3 * ncell + c], p[4 * ncell + c], H.gamma - 1.0, Wd)) {
      r.bad = 1;
      r.bad_block = std::min(r.bad_block, b);
    } else {
      r.lam = std::max(r.lam, H.ndim == 3 ? cell_rate<3>(Wd, H.gamma, d.dx[0], d.dx[1], d.dx[2])
                                          : cell_rate<2>(Wd, H.gamma, d.dx[0], d.dx[1], d.dx[2]));
    }
  }
}

}  // namespace

HostRate host_run(const HostStage &H, int nthreads, bool rate_only) {
  HostRate total;
  const int nb = (int)H.ids.size();
  if (nb == 0) return total;
  const int nt = std::max(1, std::min(nthreads, nb));
  std::atomic<int> next(0);
  std::vector<HostRate> part(nt);
  auto work = [&](int t) {
    Scratch S;
    for (int q = next.fetch_add(1); q < nb; q = next.fetch_add(1)) {
      if (rate_only)
        block_rate(H, H.ids[q], part[t]);
      else
        block_stage(H, H.ids[q], S, part[t]);
    }
  };
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
  for (const HostRate &p : part) {
    total.lam = std::max(total.lam, p.lam);
    total.bad |= p.bad;
    total.bad_block = std::min(total.bad_block, p.bad_block);
  }
  return total;
}

}  // namespace hyd
