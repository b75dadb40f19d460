"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle (on the CPU) makes at least one pin test fail.

Every mutant is one textual change of ``oracle/hydro_oracle.c`` (a dropped
term, a wrong sign, index or operand), compiled into a temporary library that
the pin tests load through ``HYDRO_ORACLE_LIB`` in a child pytest process.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hydro_oracle.c")
PINS = ["tests/test_oracle_pointwise.py", "tests/test_oracle_scheme.py", "tests/test_oracle_einfeldt.py",
        "tests/test_oracle_pvrs.py", "tests/test_oracle_recon.py", "tests/test_oracle_eos.py",
        "tests/test_oracle_bruteforce.py"]

MUTANTS = {
    "hllc-left-star-uses-SR": ("F[v] = FL[v] + SL * (Us[v] - UL[v]);", "F[v] = FL[v] + SR * (Us[v] - UL[v]);"),
    "hllc-star-energy-sign": ("(Ss + pL / (rL * (SL - uL)))", "(Ss - pL / (rL * (SL - uL)))"),
    "hllc-contact-speed-sign": ("double Ss = (pR - pL +", "double Ss = (pL - pR +"),
    "hllc-davis-drops-right": ("double SL = fmin(uL - cL, uR - cR);", "double SL = uL - cL;"),
    "hllc-energy-flux-drops-p": ("uR * (ER + pR)};", "uR * ER};"),
    "hllc-tangential-star": ("a * Ss, a * vR, a * wR,", "a * Ss, a * vL, a * wR,"),
    "plm-right-state-sign": ("wr[v] = w2 - 0.5 *", "wr[v] = w2 + 0.5 *"),
    "plm-wrong-slope-pair": ("oracle_minmod(w2 - w1, w3 - w2)", "oracle_minmod(w1 - w0, w3 - w2)"),
    "minmod-picks-larger": ("if (a > 0.0 && b > 0.0) return a < b ? a : b;", "if (a > 0.0 && b > 0.0) return a > b ? a : b;"),
    "recovery-drops-w-term": ("0.5 * (U[1] * W[1] + U[2] * W[2] + U[3] * W[3])", "0.5 * (U[1] * W[1] + U[2] * W[2])"),
    "guard-neighbour-off-by-one": ("sc = side ? layer - 1 : nsrc - layer;", "sc = side ? layer : nsrc - layer;"),
    "guard-outflow-wrong-layer": ("sc = side ? n[axis] - 1 : 0;", "sc = side ? n[axis] - 2 : 0;"),
    "rotation-not-swapped-back": ("f[1] = f[1 + d];\n          f[1 + d] = t;", "(void)t;"),
    "rk2-drops-un": ("Uout[a] = 0.5 * Un[a] + 0.5 * (src + d);", "Uout[a] = src + 0.5 * d;"),
    "cfl-uses-x-velocity": ("lam += (fabs(W[1 + d]) + c) / dx[d];", "lam += (fabs(W[1]) + c) / dx[d];"),
    "update-wrong-face": ("hi[d] += 1;", "hi[d] += 0;"),
    "einfeldt-jump-factor": ("double eta2 = 0.5 * sL * sR", "double eta2 = sL * sR"),
    "einfeldt-density-weights": ("double ubar = (sL * uL + sR * uR) / (sL + sR);",
                                 "double ubar = (rL * uL + rR * uR) / (rL + rR);"),
    "einfeldt-unweighted-c2": ("(sL * cL * cL + sR * cR * cR) / (sL + sR)", "(cL * cL + cR * cR) / 2.0"),
    "einfeldt-step-uses-davis": ("oracle_hllc_eos(rl, rr, gamma, m->speeds, m->eos, f);",
                                 "oracle_hllc_eos(rl, rr, gamma, ORACLE_SPEEDS_DAVIS, m->eos, f);"),
    "pvrs-jump-sign": ("0.5 * (pL + pR) - 0.5 * (uR - uL)", "0.5 * (pL + pR) + 0.5 * (uR - uL)"),
    "pvrs-impedance-left-only": ("double rbar = 0.5 * (rL + rR)", "double rbar = rL"),
    "pvrs-shock-factor": ("double k = (gamma + 1.0) / (2.0 * gamma);", "double k = (gamma - 1.0) / (2.0 * gamma);"),
    "pvrs-branch-inverted": ("double qR = ps <= pR ? 1.0 :", "double qR = ps >= pR ? 1.0 :"),
    "pvrs-right-uses-left-sound": ("S[1] = uR + cR * qR;", "S[1] = uR + cL * qR;"),
    "recon-conserved-uses-primitives": ("    oracle_plm_face(u, ul, ur);", "    oracle_plm_face(&w[0][0], ul, ur);"),
    "recon-no-face-state-check": ("if (!prim_ok(wl) || !prim_ok(wr)) return ORACLE_ENONPHYS;", "(void)0;"),
    "recon-right-state-from-left": ("    oracle_prim_eos(ur, gamma, eos, wr);", "    oracle_prim_eos(ul, gamma, eos, wr);"),
    "recon-option-ignored": ("face_states_eos(&u[0][0], gamma, m->recon, m->eos, d, wl, wr);",
                             "face_states_eos(&u[0][0], gamma, ORACLE_RECON_PRIMITIVE, m->eos, d, wl, wr);"),
    "char-impedance-sign": ("double ap = oracle_minmod((da[4] + rc * da[n])", "double ap = oracle_minmod((da[4] - rc * da[n])"),
    "char-entropy-drops-pressure": ("double a0 = oracle_minmod(da[0] - da[4] / c2, db[0] - db[4] / c2);",
                                    "double a0 = oracle_minmod(da[0], db[0] - db[4] / c2);"),
    "char-velocity-back-factor": ("s[n] = (c / W[0]) * (ap - am);", "s[n] = (c * W[0]) * (ap - am);"),
    "char-normal-index": ("int n = 1 + dir,", "int n = 1,"),
    "char-right-slope-cell": ("char_slope(w[2], d12, d23, gamma, dir, s2);", "char_slope(w[1], d12, d23, gamma, dir, s2);"),
    "eos-gamma1-numerator": ("(4.0 - 3.0 * beta) * (4.0 - 3.0 * beta) * g1", "(4.0 - 2.0 * beta) * (4.0 - 3.0 * beta) * g1"),
    "eos-radiation-energy-as-pressure": ("double f = cv * T + ORACLE_ARAD * T3 * T - rhoe;",
                                         "double f = cv * T + ORACLE_ARAD * T3 * T / 3.0 - rhoe;"),
    "eos-newton-derivative": ("double fp = cv + 4.0 * ORACLE_ARAD * T3;", "double fp = cv + 3.0 * ORACLE_ARAD * T3;"),
    "eos-prim-radiation-pressure": ("W[4] = U[0] * T + ORACLE_ARAD * T * T * T * T / 3.0;",
                                    "W[4] = U[0] * T + ORACLE_ARAD * T * T * T * T;"),
    "eos-sound-uses-gamma": ("*c = sqrt(oracle_gr_gamma1(W[0], T, W[4], gamma) * W[4] / W[0]);",
                             "*c = sqrt(gamma * W[4] / W[0]);"),
    "eos-step-hllc-ideal": ("oracle_hllc_eos(rl, rr, gamma, m->speeds, m->eos, f);",
                            "oracle_hllc_eos(rl, rr, gamma, m->speeds, ORACLE_EOS_IDEAL, f);"),
    "eos-cfl-ideal": ("double l = cell_lambda(w, gamma, m->eos, m->dx + 3 * b, m->ndim);",
                      "double l = cell_lambda(w, gamma, ORACLE_EOS_IDEAL, m->dx + 3 * b, m->ndim);"),
}


# The pin file written for a mutant's part of the oracle runs first, so the
# child pytest (-x) usually stops within seconds; every pin file still runs
# if that one passes, so a mutant survives only if it passes them all.
FIRST = {"eos": "tests/test_oracle_eos.py", "char": "tests/test_oracle_recon.py", "recon": "tests/test_oracle_recon.py",
         "pvrs": "tests/test_oracle_pvrs.py", "einfeldt": "tests/test_oracle_einfeldt.py"}


def pin_order(name):
    first = FIRST.get(name.split("-")[0])
    return ([first] if first else []) + [p for p in PINS if p != first]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(lib), str(mpath), "-lm"], check=True)
    env = dict(os.environ, HYDRO_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pin_order(name)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived every pin:\n{r.stdout[-2000:]}"
