/*
 * hydro_oracle.c -- plain, slow, FP64 CPU reference for one explicit
 * finite-volume compressible-Euler SSP-RK2 step on a set of mesh blocks.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The product (the HIP
 * library) never calls it, and the two share no code: this file includes no
 * header of the product and the product includes nothing from here.
 *
 * What is computed, and where it comes from
 * -----------------------------------------
 * ORCHA (arXiv 2507.09337) offloads the per-block physics task of Flash-X to
 * the GPU.  For its hydro-only Sedov application the paper states:
 *   - Sec. 5.1 (Flash-X): the domain is split into blocks that all hold the
 *     same number of equally sized cells;
 *   - Sec. 5.2 (Sedov blast wave): the only other physics is the ideal-gas
 *     gamma-law equation of state (a gas + radiation EOS, iterated like the
 *     heavier tabulated one of the paper's other application, is a method
 *     variant here);
 *   - Sec. 6 (Experiments): the hydro solver is an explicit finite-volume
 *     method whose guard cells form a halo around the block being updated,
 *     integrated with a 2nd-order Runge-Kutta method that refreshes the
 *     guard cells before each stage.
 * The paper does not spell out the reconstruction, the Riemann solver or the
 * time-step rule.  This reference fixes them to named textbook methods:
 *   - PLM (van Leer 1979) on primitive variables (rho, u, v, w, p) with the
 *     minmod limiter (Roe 1986), one direction at a time, unsplit; as
 *     method variants, PLM on the conserved variables with the face states
 *     recovered afterwards, or on the characteristic variables of the
 *     primitive system (Toro 2009, ch. 3 and sec. 14.4);
 *   - HLLC approximate Riemann solver (Toro, Spruce & Speares 1994; Toro,
 *     "Riemann Solvers and Numerical Methods for Fluid Dynamics", 3rd ed.,
 *     ch. 10) with Davis (1988) wave-speed bounds, or, as method variants,
 *     Einfeldt's (1988) bounds from Roe-weighted averages (Toro sec. 10.5.1)
 *     or pressure-based bounds (Toro sec. 10.5.2);
 *   - SSP-RK2 / TVD-RK2 (Shu & Osher 1988):
 *         U1   = Un + dt L(Un)
 *         Un+1 = 0.5 Un + 0.5 (U1 + dt L(U1));
 *   - CFL time step dt = C / max over interior cells of
 *     sum over active directions d of (|u_d| + c) / dx_d, taken from Un once
 *     per step and shared by both stages.
 * Guard cells: two layers per side.  Only the face slabs are filled (the
 * face-based unsplit stencil never reads edge or corner guards).  A face is
 * either linked to a neighbour block (copy of the neighbour's two nearest
 * interior layers), periodic on the block itself (wrap), or outflow
 * (zero-gradient copy of the first interior layer into both guard layers).
 * No floors: a non-positive density or pressure, or a non-finite value, in a
 * recovered state (a cell's, or with conserved or characteristic
 * reconstruction a face state's) is an error (ORACLE_ENONPHYS).
 *
 * Build: -O2 -ffp-contract=off -fno-fast-math, so every operation is rounded
 * as written.  OpenMP runs blocks of one stage in parallel; every block's
 * result depends only on data that is fixed during that stage, so the result
 * does not depend on the thread count.
 *
 * State layout at the interface (the "block arena"): for block b, variable v
 * (0 rho, 1 rho*u, 2 rho*v, 3 rho*w, 4 E) and interior cell (i, j, k):
 *     U[offset[b] + v * nx*ny*nz + (k*ny + j)*nx + i].
 * Internally every block is copied into its own guard-padded array.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NVAR 5
#define NG 2

enum { ORACLE_NBR = 0, ORACLE_OUTFLOW = 1, ORACLE_PERIODIC_SELF = 2 };
enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ENOMEM = 3, ORACLE_ENONPHYS = 4 };
enum { ORACLE_SPEEDS_DAVIS = 0, ORACLE_SPEEDS_EINFELDT = 1, ORACLE_SPEEDS_PVRS = 2 };
enum { ORACLE_RECON_PRIMITIVE = 0, ORACLE_RECON_CONSERVED = 1, ORACLE_RECON_CHARACTERISTIC = 2 };
enum { ORACLE_EOS_IDEAL = 0, ORACLE_EOS_GAS_RADIATION = 1 };

typedef struct {
  int32_t nblocks;
  int32_t ndim;          /* 2 or 3 */
  const int32_t *n;      /* [nblocks][3] interior cells; n[2] == 1 in 2D */
  const double *dx;      /* [nblocks][3] cell widths */
  const int32_t *kind;   /* [nblocks][6] face kind for -x,+x,-y,+y,-z,+z */
  const int32_t *nbr;    /* [nblocks][6] neighbour block id of ORACLE_NBR faces */
  const int64_t *offset; /* [nblocks] element offset of variable 0 in the arena */
  int32_t speeds;        /* HLLC wave-speed bounds: ORACLE_SPEEDS_DAVIS, _EINFELDT or _PVRS */
  int32_t recon;         /* PLM variables: ORACLE_RECON_PRIMITIVE, _CONSERVED or _CHARACTERISTIC */
  int32_t eos;           /* ORACLE_EOS_IDEAL or ORACLE_EOS_GAS_RADIATION */
} oracle_mesh;

/* ------------------------------------------------------------------------ */
/* Guard-padded copy of one block.                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n[3]; /* interior extent */
  int g[3]; /* guard width per axis: 2, or 0 on the inactive z axis in 2D */
  int p[3]; /* padded extent n + 2g */
  double *q; /* [NVAR][p2][p1][p0] */
} pblock;

static size_t pidx(const pblock *B, int v, int i, int j, int k) {
  return (((size_t)v * B->p[2] + (size_t)(k + B->g[2])) * B->p[1] + (size_t)(j + B->g[1])) * B->p[0] +
         (size_t)(i + B->g[0]);
}

static size_t aidx(const oracle_mesh *m, int b, int v, int i, int j, int k) {
  const int32_t *n = m->n + 3 * b;
  return (size_t)m->offset[b] + (size_t)v * n[0] * n[1] * n[2] + ((size_t)k * n[1] + j) * n[0] + i;
}

static int pblock_alloc(pblock *B, const oracle_mesh *m, int b) {
  for (int d = 0; d < 3; ++d) {
    B->n[d] = m->n[3 * b + d];
    B->g[d] = (d < m->ndim) ? NG : 0;
    B->p[d] = B->n[d] + 2 * B->g[d];
  }
  size_t len = (size_t)NVAR * B->p[0] * B->p[1] * B->p[2];
  B->q = (double *)malloc(len * sizeof(double));
  if (!B->q) return ORACLE_ENOMEM;
  /* Edge and corner guards are never filled; NaN makes any read of them loud. */
  for (size_t s = 0; s < len; ++s) B->q[s] = NAN;
  return ORACLE_OK;
}

/*
 * Copy block b of the arena into B and fill the two guard layers of every
 * face slab (Sec. 6: guard cells form a halo; refreshed before each stage).
 */
static void pblock_load(pblock *B, const oracle_mesh *m, int b, const double *U) {
  const int *n = B->n;
  for (int v = 0; v < NVAR; ++v)
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) B->q[pidx(B, v, i, j, k)] = U[aidx(m, b, v, i, j, k)];

  for (int axis = 0; axis < m->ndim; ++axis) {
    for (int side = 0; side < 2; ++side) {
      int face = 2 * axis + side;
      int kind = m->kind[6 * b + face];
      int src = (kind == ORACLE_NBR) ? m->nbr[6 * b + face] : b;
      int nsrc = m->n[3 * src + axis];
      for (int layer = 1; layer <= NG; ++layer) {
        /* guard coordinate along the axis, and the source coordinate in block src */
        int gc = side ? n[axis] - 1 + layer : -layer;
        int sc;
        if (kind == ORACLE_OUTFLOW)
          sc = side ? n[axis] - 1 : 0;
        else /* neighbour or periodic wrap: the far side of the source block */
          sc = side ? layer - 1 : nsrc - layer;
        for (int v = 0; v < NVAR; ++v)
          for (int k = 0; k < (axis == 2 ? 1 : n[2]); ++k)
            for (int j = 0; j < (axis == 1 ? 1 : n[1]); ++j)
              for (int i = 0; i < (axis == 0 ? 1 : n[0]); ++i) {
                int d[3] = {i, j, k}, s[3] = {i, j, k};
                d[axis] = gc;
                s[axis] = sc;
                B->q[pidx(B, v, d[0], d[1], d[2])] = U[aidx(m, src, v, s[0], s[1], s[2])];
              }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Pointwise physics.                                                        */
/* ------------------------------------------------------------------------ */

/* Conserved -> primitive with the ideal-gas gamma-law EOS (Sec. 5.2):
 * u_d = m_d / rho;  rho*e = E - (m_x u + m_y v + m_z w)/2;  p = (gamma-1) rho*e. */
static double velocities_and_rhoe(const double *U, double *W) {
  W[0] = U[0];
  W[1] = U[1] / U[0];
  W[2] = U[2] / U[0];
  W[3] = U[3] / U[0];
  return U[4] - 0.5 * (U[1] * W[1] + U[2] * W[2] + U[3] * W[3]);
}

void oracle_prim(const double *U, double gamma, double *W) {
  double rhoe = velocities_and_rhoe(U, W);
  W[4] = (gamma - 1.0) * rhoe;
}

static int prim_ok(const double *W) {
  for (int v = 0; v < NVAR; ++v)
    if (!isfinite(W[v])) return 0;
  return W[0] > 0.0 && W[4] > 0.0;
}

/*
 * Gas + radiation equation of state, a method variant standing in for a
 * heavier (iterated) EOS: an ideal gas of adiabatic index gamma in
 * equilibrium with black-body radiation, in units where the gas constant and
 * the radiation constant are 1:
 *     p = rho T + T^4 / 3,        rho e = rho T / (gamma - 1) + T^4.
 * The temperature is the root of a convex increasing quartic, found by
 * Newton's method from an upper bound (the smaller of the gas-only and the
 * radiation-only temperature), so the iterates decrease monotonically; the
 * iteration stops when an iterate no longer decreases.  The sound speed is
 * c^2 = Gamma1 p / rho with the first adiabatic exponent of the mixture
 * (Clayton 1968), beta = rho T / p the gas share of the pressure:
 *     Gamma1 = beta + (4 - 3 beta)^2 (gamma - 1) / (beta + 12 (gamma - 1)(1 - beta)).
 */
#define ORACLE_ARAD 1.0

double oracle_gr_temperature_e(double rho, double rhoe, double gamma) {
  double cv = rho / (gamma - 1.0); /* rho c_v */
  double T = fmin(rhoe / cv, sqrt(sqrt(rhoe / ORACLE_ARAD)));
  for (int k = 0; k < 64; ++k) {
    double T3 = T * T * T;
    double f = cv * T + ORACLE_ARAD * T3 * T - rhoe;
    double fp = cv + 4.0 * ORACLE_ARAD * T3;
    double Tn = T - f / fp;
    if (!(Tn < T)) break;
    T = Tn;
  }
  return T;
}

double oracle_gr_temperature_p(double rho, double p) {
  double T = fmin(p / rho, sqrt(sqrt(3.0 * p / ORACLE_ARAD)));
  for (int k = 0; k < 64; ++k) {
    double T3 = T * T * T;
    double f = rho * T + ORACLE_ARAD * T3 * T / 3.0 - p;
    double fp = rho + 4.0 * ORACLE_ARAD * T3 / 3.0;
    double Tn = T - f / fp;
    if (!(Tn < T)) break;
    T = Tn;
  }
  return T;
}

double oracle_gr_gamma1(double rho, double T, double p, double gamma) {
  double beta = rho * T / p;
  double g1 = gamma - 1.0;
  return beta + (4.0 - 3.0 * beta) * (4.0 - 3.0 * beta) * g1 / (beta + 12.0 * g1 * (1.0 - beta));
}

/* Conserved -> primitive under either EOS (the ideal one is oracle_prim).
 * Gas + radiation: p from the temperature of rho e = E - m.u/2; a state with
 * rho e <= 0 has no temperature and gets p = rho e (non-physical). */
void oracle_prim_eos(const double *U, double gamma, int eos, double *W) {
  if (eos != ORACLE_EOS_GAS_RADIATION) {
    oracle_prim(U, gamma, W);
    return;
  }
  double rhoe = velocities_and_rhoe(U, W);
  if (!(rhoe > 0.0)) {
    W[4] = rhoe;
    return;
  }
  double T = oracle_gr_temperature_e(U[0], rhoe, gamma);
  W[4] = U[0] * T + ORACLE_ARAD * T * T * T * T / 3.0;
}

/* Sound speed and internal energy per volume of primitive state W. */
void oracle_thermo(const double *W, double gamma, int eos, double *c, double *rhoe) {
  if (eos == ORACLE_EOS_GAS_RADIATION) {
    double T = oracle_gr_temperature_p(W[0], W[4]);
    *c = sqrt(oracle_gr_gamma1(W[0], T, W[4], gamma) * W[4] / W[0]);
    *rhoe = W[0] * T / (gamma - 1.0) + ORACLE_ARAD * T * T * T * T;
  } else {
    *c = sqrt(gamma * W[4] / W[0]);
    *rhoe = W[4] / (gamma - 1.0);
  }
}

/* minmod limiter (Roe 1986): the argument of smaller magnitude when both have
 * the same strict sign, else zero.  Signs are tested directly (no a*b). */
double oracle_minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* PLM face states at the face between cells 1 and 2 of four consecutive
 * cells w[0..3] along one direction (van Leer 1979, limited by minmod):
 *   left  state  = w1 + minmod(w1 - w0, w2 - w1) / 2
 *   right state  = w2 - minmod(w2 - w1, w3 - w2) / 2
 * w is [4][NVAR]; wl, wr are [NVAR]. */
void oracle_plm_face(const double *w, double *wl, double *wr) {
  for (int v = 0; v < NVAR; ++v) {
    double w0 = w[0 * NVAR + v], w1 = w[1 * NVAR + v], w2 = w[2 * NVAR + v], w3 = w[3 * NVAR + v];
    wl[v] = w1 + 0.5 * oracle_minmod(w1 - w0, w2 - w1);
    wr[v] = w2 - 0.5 * oracle_minmod(w2 - w1, w3 - w2);
  }
}

/* Limited slope of cell W (primitives) on the characteristic variables of
 * the primitive Euler system along direction `dir` (Toro 2009, ch. 3: the
 * system W_t + A W_x = 0 with normal velocity u_n = W[1 + dir], waves
 * u_n - c, u_n (entropy and two shear waves), u_n + c), from the one-sided
 * differences da = W - W_left and db = W_right - W:
 *   amplitudes of a difference d (left eigenvectors at W, rho c = impedance):
 *     a_-  = (d_p - rho c d_un) / (2 c^2),   a_0 = d_rho - d_p / c^2,
 *     a_t1 = d_ut1,  a_t2 = d_ut2,           a_+ = (d_p + rho c d_un) / (2 c^2);
 *   each amplitude limited by minmod of its two one-sided values, m_k;
 *   slope = sum_k m_k r_k with the right eigenvectors at W:
 *     d_rho = m_- + m_0 + m_+,  d_un = (c / rho)(m_+ - m_-),
 *     d_ut = m_t,               d_p  = c^2 (m_- + m_+). */
static void char_slope(const double *W, const double *da, const double *db, double gamma, int dir, double *s) {
  int n = 1 + dir, t1 = 1 + (dir + 1) % 3, t2 = 1 + (dir + 2) % 3;
  double c = sqrt(gamma * W[4] / W[0]);
  double rc = W[0] * c, c2 = c * c;
  double am = oracle_minmod((da[4] - rc * da[n]) / (2.0 * c2), (db[4] - rc * db[n]) / (2.0 * c2));
  double a0 = oracle_minmod(da[0] - da[4] / c2, db[0] - db[4] / c2);
  double at1 = oracle_minmod(da[t1], db[t1]);
  double at2 = oracle_minmod(da[t2], db[t2]);
  double ap = oracle_minmod((da[4] + rc * da[n]) / (2.0 * c2), (db[4] + rc * db[n]) / (2.0 * c2));
  s[0] = am + a0 + ap;
  s[n] = (c / W[0]) * (ap - am);
  s[t1] = at1;
  s[t2] = at2;
  s[4] = c2 * (am + ap);
}

/* Primitive face states at the face between cells 1 and 2 of four
 * consecutive cells along direction dir (0 x, 1 y, 2 z) given by their
 * conserved values u[0..3] ([4][NVAR]).  Every cell's primitives are
 * recovered first (a non-physical cell is an error).  Then PLM runs on the
 * variables `recon` names:
 *   ORACLE_RECON_PRIMITIVE: on the recovered (rho, u, v, w, p);
 *   ORACLE_RECON_CONSERVED: on (rho, rho u, rho v, rho w, E) themselves
 *     (van Leer's MUSCL on the conserved variables), after which the two face
 *     states are recovered with the same formulas;
 *   ORACLE_RECON_CHARACTERISTIC: on the characteristic variables of each of
 *     the two cells (char_slope): left state W_1 + slope_1 / 2, right state
 *     W_2 - slope_2 / 2.
 * With the last two a non-physical face state (rho <= 0, p <= 0,
 * non-finite) is an error as well.  Returns ORACLE_OK or ORACLE_ENONPHYS. */
static int face_states_eos(const double *u, double gamma, int recon, int eos, int dir, double *wl, double *wr) {
  double w[4][NVAR];
  for (int s = 0; s < 4; ++s) {
    oracle_prim_eos(u + s * NVAR, gamma, eos, w[s]);
    if (!prim_ok(w[s])) return ORACLE_ENONPHYS;
  }
  if (recon == ORACLE_RECON_CONSERVED) {
    double ul[NVAR], ur[NVAR];
    oracle_plm_face(u, ul, ur);
    oracle_prim_eos(ul, gamma, eos, wl);
    oracle_prim_eos(ur, gamma, eos, wr);
  } else if (recon == ORACLE_RECON_CHARACTERISTIC) {
    double d01[NVAR], d12[NVAR], d23[NVAR], s1[NVAR], s2[NVAR];
    for (int v = 0; v < NVAR; ++v) {
      d01[v] = w[1][v] - w[0][v];
      d12[v] = w[2][v] - w[1][v];
      d23[v] = w[3][v] - w[2][v];
    }
    char_slope(w[1], d01, d12, gamma, dir, s1);
    char_slope(w[2], d12, d23, gamma, dir, s2);
    for (int v = 0; v < NVAR; ++v) {
      wl[v] = w[1][v] + 0.5 * s1[v];
      wr[v] = w[2][v] - 0.5 * s2[v];
    }
  } else {
    oracle_plm_face(&w[0][0], wl, wr);
    return ORACLE_OK;
  }
  if (!prim_ok(wl) || !prim_ok(wr)) return ORACLE_ENONPHYS;
  return ORACLE_OK;
}

int oracle_face_states(const double *u, double gamma, int recon, int dir, double *wl, double *wr) {
  return face_states_eos(u, gamma, recon, ORACLE_EOS_IDEAL, dir, wl, wr);
}

/*
 * Bounds S = (S_L, S_R) of the wave speeds of the Riemann problem at a face
 * whose normal is the first velocity component, c_K = sqrt(gamma p_K / rho_K).
 *   Davis (1988):     S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).
 *   Einfeldt (1988), as stated in Toro (2009) sec. 10.5.1:
 *     with s_K = sqrt(rho_K), the Roe-weighted normal velocity
 *       u_bar = (s_L u_L + s_R u_R) / (s_L + s_R),
 *     d_bar^2 = (s_L c_L^2 + s_R c_R^2) / (s_L + s_R) + eta2 (u_R - u_L)^2,
 *       eta2 = s_L s_R / (2 (s_L + s_R)^2),
 *     S_L = u_bar - d_bar, S_R = u_bar + d_bar.
 *   Pressure-based (Toro 2009, sec. 10.5.2) with the primitive-variable
 *   (PVRS) estimate of the star pressure:
 *     p_pvrs = (p_L + p_R)/2 - (u_R - u_L) rho_bar c_bar / 2,
 *       rho_bar = (rho_L + rho_R)/2, c_bar = (c_L + c_R)/2,  p* = max(0, p_pvrs);
 *     q_K = 1 if p* <= p_K (a rarefaction: the acoustic speed), else the
 *       shock factor q_K = sqrt(1 + (gamma + 1)/(2 gamma) (p* / p_K - 1));
 *     S_L = u_L - c_L q_L, S_R = u_R + c_R q_R.
 */
static void wave_speeds_c(const double *WL, const double *WR, double cL, double cR, double gamma, int speeds,
                          double *S) {
  double rL = WL[0], uL = WL[1], pL = WL[4];
  double rR = WR[0], uR = WR[1], pR = WR[4];
  if (speeds == ORACLE_SPEEDS_EINFELDT) {
    double sL = sqrt(rL), sR = sqrt(rR);
    double ubar = (sL * uL + sR * uR) / (sL + sR);
    double eta2 = 0.5 * sL * sR / ((sL + sR) * (sL + sR));
    double dbar = sqrt((sL * cL * cL + sR * cR * cR) / (sL + sR) + eta2 * (uR - uL) * (uR - uL));
    S[0] = ubar - dbar;
    S[1] = ubar + dbar;
  } else if (speeds == ORACLE_SPEEDS_PVRS) {
    double rbar = 0.5 * (rL + rR), cbar = 0.5 * (cL + cR);
    double ppv = 0.5 * (pL + pR) - 0.5 * (uR - uL) * rbar * cbar;
    double ps = fmax(0.0, ppv);
    double k = (gamma + 1.0) / (2.0 * gamma);
    double qL = ps <= pL ? 1.0 : sqrt(1.0 + k * (ps / pL - 1.0));
    double qR = ps <= pR ? 1.0 : sqrt(1.0 + k * (ps / pR - 1.0));
    S[0] = uL - cL * qL;
    S[1] = uR + cR * qR;
  } else {
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    S[0] = SL;
    S[1] = SR;
  }
}

void oracle_wave_speeds(const double *WL, const double *WR, double gamma, int speeds, double *S) {
  double cL = sqrt(gamma * WL[4] / WL[0]);
  double cR = sqrt(gamma * WR[4] / WR[0]);
  wave_speeds_c(WL, WR, cL, cR, gamma, speeds, S);
}

/*
 * HLLC flux across a face whose normal is the first velocity component
 * (Toro 2009, sec. 10.4-10.6; Toro, Spruce & Speares 1994).
 * WL, WR = (rho, u_normal, u_t1, u_t2, p).  F = (mass, normal momentum,
 * t1 momentum, t2 momentum, energy) flux in the same frame.
 *   Wave speeds S_L, S_R: oracle_wave_speeds (Davis, Einfeldt or PVRS), with
 *   the sound speeds and E_K = rho e_K + rho_K |v_K|^2 / 2 of the EOS
 *   (oracle_thermo).
 *   Contact speed: S* = [p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R)]
 *                       / [rho_L (S_L - u_L) - rho_R (S_R - u_R)].
 *   Star states:   U*_K = rho_K (S_K - u_K)/(S_K - S*) *
 *                  (1, S*, v_K, w_K, E_K/rho_K + (S* - u_K)(S* + p_K/(rho_K (S_K - u_K)))).
 *   Flux:  F_L                    if 0 <= S_L
 *          F_L + S_L (U*_L - U_L) if S_L < 0 <= S*
 *          F_R + S_R (U*_R - U_R) if S* < 0 < S_R
 *          F_R                    if S_R <= 0.
 */
void oracle_hllc_eos(const double *WL, const double *WR, double gamma, int speeds, int eos, double *F) {
  double rL = WL[0], uL = WL[1], vL = WL[2], wL = WL[3], pL = WL[4];
  double rR = WR[0], uR = WR[1], vR = WR[2], wR = WR[3], pR = WR[4];
  double cL, cR, eL, eR;
  oracle_thermo(WL, gamma, eos, &cL, &eL);
  oracle_thermo(WR, gamma, eos, &cR, &eR);
  double EL = eL + 0.5 * rL * (uL * uL + vL * vL + wL * wL);
  double ER = eR + 0.5 * rR * (uR * uR + vR * vR + wR * wR);

  double S[2];
  wave_speeds_c(WL, WR, cL, cR, gamma, speeds, S);
  double SL = S[0], SR = S[1];
  double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR));

  double UL[NVAR] = {rL, rL * uL, rL * vL, rL * wL, EL};
  double UR[NVAR] = {rR, rR * uR, rR * vR, rR * wR, ER};
  double FL[NVAR] = {rL * uL, rL * uL * uL + pL, rL * uL * vL, rL * uL * wL, uL * (EL + pL)};
  double FR[NVAR] = {rR * uR, rR * uR * uR + pR, rR * uR * vR, rR * uR * wR, uR * (ER + pR)};

  if (0.0 <= SL) {
    for (int v = 0; v < NVAR; ++v) F[v] = FL[v];
  } else if (0.0 <= Ss) {
    double a = rL * (SL - uL) / (SL - Ss);
    double Us[NVAR] = {a, a * Ss, a * vL, a * wL, a * (EL / rL + (Ss - uL) * (Ss + pL / (rL * (SL - uL))))};
    for (int v = 0; v < NVAR; ++v) F[v] = FL[v] + SL * (Us[v] - UL[v]);
  } else if (0.0 < SR) {
    double a = rR * (SR - uR) / (SR - Ss);
    double Us[NVAR] = {a, a * Ss, a * vR, a * wR, a * (ER / rR + (Ss - uR) * (Ss + pR / (rR * (SR - uR))))};
    for (int v = 0; v < NVAR; ++v) F[v] = FR[v] + SR * (Us[v] - UR[v]);
  } else {
    for (int v = 0; v < NVAR; ++v) F[v] = FR[v];
  }
}

/* HLLC with the ideal-gas EOS. */
void oracle_hllc_speeds(const double *WL, const double *WR, double gamma, int speeds, double *F) {
  oracle_hllc_eos(WL, WR, gamma, speeds, ORACLE_EOS_IDEAL, F);
}

/* HLLC with Davis wave speeds. */
void oracle_hllc(const double *WL, const double *WR, double gamma, double *F) {
  oracle_hllc_speeds(WL, WR, gamma, ORACLE_SPEEDS_DAVIS, F);
}

/* Local CFL rate of one cell: sum over active directions of (|u_d| + c)/dx_d. */
static double cell_lambda(const double *W, double gamma, int eos, const double *dx, int ndim) {
  double c, rhoe;
  oracle_thermo(W, gamma, eos, &c, &rhoe);
  double lam = 0.0;
  for (int d = 0; d < ndim; ++d) lam += (fabs(W[1 + d]) + c) / dx[d];
  return lam;
}

/* ------------------------------------------------------------------------ */
/* One RK stage of one block.                                                */
/* ------------------------------------------------------------------------ */

/*
 * Stage of block b:  dU = sum over active d of (dt/dx_d)(F_{d,lo face} - F_{d,hi face})
 * summed in x, y, z order, with F from PLM + HLLC on the guard-filled source state.
 *   stage 1:  Uout = Usrc + dU                      (Usrc = Un)
 *   stage 2:  Uout = 0.5 Un + 0.5 (Usrc + dU)       (Usrc = U1)
 * Reads Usrc for block b and its face neighbours, Un for block b only; writes
 * block b of Uout (which may alias Un).
 */
static int block_stage(const oracle_mesh *m, int b, const double *Usrc, const double *Un, double dt, double gamma,
                       int stage, double *Uout) {
  pblock S;
  int rc = pblock_alloc(&S, m, b);
  if (rc) return rc;
  pblock_load(&S, m, b, Usrc);

  const int *n = S.n;
  const double *dx = m->dx + 3 * b;
  size_t ncell = (size_t)n[0] * n[1] * n[2];
  double *dU = (double *)calloc(NVAR * ncell, sizeof(double));
  /* flux on the n+1 faces of every line of every active direction */
  size_t nface_max = (size_t)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  double *flux = (double *)malloc(NVAR * nface_max * sizeof(double));
  if (!dU || !flux) {
    free(S.q);
    free(dU);
    free(flux);
    return ORACLE_ENOMEM;
  }
  rc = ORACLE_OK;

  for (int d = 0; d < m->ndim && rc == ORACLE_OK; ++d) {
    int fn[3] = {n[0], n[1], n[2]};
    fn[d] += 1; /* faces along d: index f in 0..n_d, face f lies between cells f-1 and f */
    for (int k = 0; k < fn[2] && rc == ORACLE_OK; ++k)
      for (int j = 0; j < fn[1] && rc == ORACLE_OK; ++j)
        for (int i = 0; i < fn[0] && rc == ORACLE_OK; ++i) {
          double u[4][NVAR];
          for (int s = 0; s < 4; ++s) {
            int c[3] = {i, j, k};
            c[d] += s - 2; /* cells f-2, f-1, f, f+1 */
            for (int v = 0; v < NVAR; ++v) u[s][v] = S.q[pidx(&S, v, c[0], c[1], c[2])];
          }
          double wl[NVAR], wr[NVAR], rl[NVAR], rr[NVAR], f[NVAR];
          rc = face_states_eos(&u[0][0], gamma, m->recon, m->eos, d, wl, wr);
          if (rc) break;
          /* rotate: the normal velocity component goes into slot 1 */
          for (int v = 0; v < NVAR; ++v) {
            rl[v] = wl[v];
            rr[v] = wr[v];
          }
          rl[1] = wl[1 + d];
          rl[1 + d] = wl[1];
          rr[1] = wr[1 + d];
          rr[1 + d] = wr[1];
          oracle_hllc_eos(rl, rr, gamma, m->speeds, m->eos, f);
          /* rotate back */
          double t = f[1];
          f[1] = f[1 + d];
          f[1 + d] = t;
          size_t fi = ((size_t)k * fn[1] + j) * fn[0] + i;
          for (int v = 0; v < NVAR; ++v) flux[(size_t)v * nface_max + fi] = f[v];
        }
    if (rc) break;
    double dtdx = dt / dx[d];
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) {
          int hi[3] = {i, j, k};
          hi[d] += 1;
          size_t flo = ((size_t)k * fn[1] + j) * fn[0] + i;
          size_t fhi = ((size_t)hi[2] * fn[1] + hi[1]) * fn[0] + hi[0];
          size_t c = ((size_t)k * n[1] + j) * n[0] + i;
          for (int v = 0; v < NVAR; ++v)
            dU[(size_t)v * ncell + c] += dtdx * (flux[(size_t)v * nface_max + flo] - flux[(size_t)v * nface_max + fhi]);
        }
  }

  if (rc == ORACLE_OK) {
    for (int v = 0; v < NVAR; ++v)
      for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
          for (int i = 0; i < n[0]; ++i) {
            size_t c = ((size_t)k * n[1] + j) * n[0] + i;
            double src = S.q[pidx(&S, v, i, j, k)];
            double d = dU[(size_t)v * ncell + c];
            size_t a = aidx(m, b, v, i, j, k);
            if (stage == 1)
              Uout[a] = src + d;
            else
              Uout[a] = 0.5 * Un[a] + 0.5 * (src + d);
          }
  }
  free(S.q);
  free(dU);
  free(flux);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Mesh-level entry points.                                                  */
/* ------------------------------------------------------------------------ */

int oracle_validate(const oracle_mesh *m) {
  if (!m || m->nblocks < 0 || (m->ndim != 2 && m->ndim != 3)) return ORACLE_EINVAL;
  if (m->nblocks > 0 && (!m->n || !m->dx || !m->kind || !m->nbr || !m->offset)) return ORACLE_EINVAL;
  if (m->speeds < ORACLE_SPEEDS_DAVIS || m->speeds > ORACLE_SPEEDS_PVRS) return ORACLE_EINVAL;
  if (m->recon < ORACLE_RECON_PRIMITIVE || m->recon > ORACLE_RECON_CHARACTERISTIC) return ORACLE_EINVAL;
  if (m->eos != ORACLE_EOS_IDEAL && m->eos != ORACLE_EOS_GAS_RADIATION) return ORACLE_EINVAL;
  /* the wave-speed and reconstruction variants assume the gamma-law EOS */
  if (m->eos == ORACLE_EOS_GAS_RADIATION && (m->speeds != ORACLE_SPEEDS_DAVIS || m->recon != ORACLE_RECON_PRIMITIVE))
    return ORACLE_EINVAL;
  for (int b = 0; b < m->nblocks; ++b) {
    const int32_t *n = m->n + 3 * b;
    if (m->ndim == 2 && n[2] != 1) return ORACLE_EINVAL;
    for (int d = 0; d < m->ndim; ++d) {
      if (n[d] < NG) return ORACLE_EINVAL;
      if (!(m->dx[3 * b + d] > 0.0)) return ORACLE_EINVAL;
    }
    if (m->offset[b] < 0) return ORACLE_EINVAL;
    for (int f = 0; f < 2 * m->ndim; ++f) {
      int kind = m->kind[6 * b + f];
      if (kind != ORACLE_NBR && kind != ORACLE_OUTFLOW && kind != ORACLE_PERIODIC_SELF) return ORACLE_EINVAL;
      if (kind == ORACLE_NBR) {
        int s = m->nbr[6 * b + f];
        if (s < 0 || s >= m->nblocks) return ORACLE_EINVAL;
        for (int d = 0; d < 3; ++d)
          if (d != f / 2 && m->n[3 * s + d] != n[d]) return ORACLE_EINVAL;
        if (m->n[3 * s + f / 2] < NG) return ORACLE_EINVAL;
      }
    }
  }
  return ORACLE_OK;
}

/* max over interior cells of all blocks of the local CFL rate; ENONPHYS if any
 * recovered state is not physical. */
int oracle_max_lambda(const oracle_mesh *m, const double *U, double gamma, double *lam_out) {
  int rc = oracle_validate(m);
  if (rc) return rc;
  double lam = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(max : lam) reduction(| : bad)
  for (int b = 0; b < m->nblocks; ++b) {
    const int32_t *n = m->n + 3 * b;
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) {
          double u[NVAR], w[NVAR];
          for (int v = 0; v < NVAR; ++v) u[v] = U[aidx(m, b, v, i, j, k)];
          oracle_prim_eos(u, gamma, m->eos, w);
          if (!prim_ok(w)) {
            bad = 1;
            continue;
          }
          double l = cell_lambda(w, gamma, m->eos, m->dx + 3 * b, m->ndim);
          if (l > lam) lam = l;
        }
  }
  if (bad) return ORACLE_ENONPHYS;
  *lam_out = lam;
  return ORACLE_OK;
}

static size_t arena_len(const oracle_mesh *m) {
  size_t len = 0;
  for (int b = 0; b < m->nblocks; ++b) {
    const int32_t *n = m->n + 3 * b;
    size_t end = (size_t)m->offset[b] + (size_t)NVAR * n[0] * n[1] * n[2];
    if (end > len) len = end;
  }
  return len;
}

/*
 * One SSP-RK2 step for the blocks listed in `targets`, reading the full state
 * Uin of every block and writing the new state of the target blocks into Uout
 * (arena layout; may equal Uin).  Stage 1 runs on the targets and on their
 * linked face neighbours, whose stage-1 values fill the targets' guards for
 * stage 2.  With targets = all blocks this is the whole-mesh step.
 */
int oracle_step_subset(const oracle_mesh *m, const double *Uin, double dt, double gamma, const int32_t *targets,
                       int32_t ntargets, double *Uout) {
  int rc = oracle_validate(m);
  if (rc) return rc;
  for (int t = 0; t < ntargets; ++t)
    if (targets[t] < 0 || targets[t] >= m->nblocks) return ORACLE_EINVAL;

  char *in1 = (char *)calloc((size_t)m->nblocks + 1, 1);
  double *U1 = (double *)calloc(arena_len(m) + 1, sizeof(double));
  if (!in1 || !U1) {
    free(in1);
    free(U1);
    return ORACLE_ENOMEM;
  }
  for (int t = 0; t < ntargets; ++t) {
    int b = targets[t];
    in1[b] = 1;
    for (int f = 0; f < 2 * m->ndim; ++f)
      if (m->kind[6 * b + f] == ORACLE_NBR) in1[m->nbr[6 * b + f]] = 1;
  }
  int32_t *list1 = (int32_t *)malloc(((size_t)m->nblocks + 1) * sizeof(int32_t));
  int n1 = 0;
  if (!list1) {
    free(in1);
    free(U1);
    return ORACLE_ENOMEM;
  }
  for (int b = 0; b < m->nblocks; ++b)
    if (in1[b]) list1[n1++] = b;

  int err = ORACLE_OK;
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < n1; ++t) {
    int e = block_stage(m, list1[t], Uin, Uin, dt, gamma, 1, U1);
    if (e) {
#pragma omp critical
      err = err ? err : e;
    }
  }
  if (err == ORACLE_OK) {
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < ntargets; ++t) {
      int e = block_stage(m, targets[t], U1, Uin, dt, gamma, 2, Uout);
      if (e) {
#pragma omp critical
        err = err ? err : e;
      }
    }
  }
  free(in1);
  free(U1);
  free(list1);
  return err;
}

/* One SSP-RK2 step of the whole mesh, in place. */
int oracle_step(const oracle_mesh *m, double *U, double dt, double gamma) {
  int rc = oracle_validate(m);
  if (rc) return rc;
  int32_t *all = (int32_t *)malloc(((size_t)m->nblocks + 1) * sizeof(int32_t));
  if (!all) return ORACLE_ENOMEM;
  for (int b = 0; b < m->nblocks; ++b) all[b] = b;
  rc = oracle_step_subset(m, U, dt, gamma, all, m->nblocks, U);
  free(all);
  return rc;
}

/*
 * nsteps steps in place.  dt = cfl / max lambda(Un) each step, or fixed_dt
 * when fixed_dt > 0.  The dt of every step goes to dts (if not NULL); the
 * elapsed time to *t_out (if not NULL).
 */
int oracle_run(const oracle_mesh *m, double *U, int32_t nsteps, double cfl, double gamma, double fixed_dt,
               double *dts, double *t_out) {
  double t = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    double dt = fixed_dt;
    if (!(fixed_dt > 0.0)) {
      double lam;
      int rc = oracle_max_lambda(m, U, gamma, &lam);
      if (rc) return rc;
      dt = cfl / lam;
    }
    int rc = oracle_step(m, U, dt, gamma);
    if (rc) return rc;
    if (dts) dts[s] = dt;
    t += dt;
  }
  if (t_out) *t_out = t;
  return ORACLE_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
