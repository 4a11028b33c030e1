"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's source (on the CPU),
compiles it, and runs the pin suite against the planted copy: at least one
pin must fail. The mistakes are the misreadings the paper's garbled formulas
invite (literal eqs. 20, 24, 26, 30, (g h)^2/2 walls) and ordinary slips
(a sign, an exponent, a swapped operand, a dropped term).
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_flux.py", "tests/test_oracle_cell.py",
        "tests/test_oracle_scheme.py", "tests/test_oracle_monitors.py"]

PLANTED = {
    # eq. 30 as printed: g instead of g/2 in the bed-slope term
    "bed_slope_factor_g": ("double pL = 0.5 * g * (hLs * hLs - hi * hi);",
                           "double pL = g * (hLs * hLs - hi * hi);"),
    # flux on the cell states instead of the reconstructed ones (eq. 37)
    "no_reconstruction": ("             hLs, ui * nx + vi * ny,",
                          "             hi, ui * nx + vi * ny,"),
    # eq. 24 as printed: downwind tangential velocity
    "downwind_tangential": ("G[2] = G[0] * (Ss >= 0.0 ? vL : vR);",
                            "G[2] = G[0] * (Ss >= 0.0 ? vR : vL);"),
    # eq. 20 as printed: /2 instead of /h_k
    "wave_factor_half": ("return sqrt(hs * (hs + hk) / 2.0) / hk;",
                         "return sqrt(hs * (hs + hk) / 2.0) / 2.0;"),
    # eq. 21 sign slip
    "pvrs_sign": ("double h0 = 0.5 * (hL + hR) - (uR - uL)",
                  "double h0 = 0.5 * (hL + hR) + (uR - uL)"),
    # eq. 23 sign slip
    "tsrs_sign": ("hs = (hL * gL + hR * gR + uL - uR) / (gL + gR);",
                  "hs = (hL * gL + hR * gR - uL + uR) / (gL + gR);"),
    # eq. 22 without the vacuum clamp
    "trrs_no_clamp": ("if (b < 0.0) b = 0.0;", ";"),
    # eq. 26, right-dry line with the rarefaction speed of a wet side
    "dry_front_speed": ("*SR = uL + 2.0 * aL;", "*SR = uL + aL;"),
    # eq. 35 with the exponent of eq. 5 (4/3) instead of 7/3
    "jacobian_exponent": ("double jhx = (7.0 / 3.0) * c * qn * hu * rh;",
                          "double jhx = (4.0 / 3.0) * c * qn * hu * rh;"),
    # friction fully explicit (no [I - dt/2 J]^-1)
    "explicit_friction": ("double m11 = 1.0 - 0.5 * dt * jxx;",
                          "double m11 = 1.0;"),
    # h^(4/3) instead of h^(7/3) in the friction coefficient
    "friction_exponent": ("double c = g * m * m / (h * h * cbrt(h));",
                          "double c = g * m * m / (h * cbrt(h));"),
    # back-rotation sign slip (eq. 12)
    "rotation_sign": ("F[1] = G[1] * nx - G[2] * ny;",
                      "F[1] = G[1] * nx + G[2] * ny;"),
    # wall pressure as printed, (g h)^2 / 2
    "wall_gh_squared": ("        G[1] = 0.5 * g * hi * hi;\n        G[2] = 0.0;\n"
                        "        break;\n    }",
                        "        G[1] = 0.5 * g * g * hi * hi;\n"
                        "        G[2] = 0.0;\n        break;\n    }"),
    # reflective wall: HLLC against the mirror state instead of the
    # hydrostatic pressure alone (reading R11)
    "wall_mirror_riemann": ("        G[0] = 0.0;\n        G[1] = 0.5 * g * hi * hi;\n"
                            "        G[2] = 0.0;\n        break;\n    }",
                            "        ora_hllc(g, h_dry, hi, un, ut, hi, -un, ut, G);\n"
                            "        break;\n    }"),
    # wall passing the momentum carried into it as well
    "wall_convective": ("        G[1] = 0.5 * g * hi * hi;\n        G[2] = 0.0;\n"
                        "        break;\n    }",
                        "        G[1] = 0.5 * g * hi * hi + hi * un * un;\n"
                        "        G[2] = 0.0;\n        break;\n    }"),
    # inflow entering with the outward sign
    "inflow_sign": ("G[0] = -q;", "G[0] = q;"),
    # diameter-free inscribed radius slip, A / perimeter
    "inradius": ("o->inr[c] = 2.0 * o->area[c] / per;",
                 "o->inr[c] = o->area[c] / per;"),
    # positivity ledger with the wrong sign
    "ledger_sign": ("*clamp = -A * hn;", "*clamp = A * hn;"),
    # a cell picks up the other side's contribution
    "wrong_side": ("const double *c = o->c_right[3 * i + k] ? &o->cr[3 * e]",
                   "const double *c = !o->c_right[3 * i + k] ? &o->cr[3 * e]"),
    # velocity of the right cell taken from the left one
    "velocity_index": ("velocity(h_dry, hj, huj, hvj, &uj, &vj);",
                       "velocity(h_dry, hi, huj, hvj, &uj, &vj);"),
    # fixed depth: ghost placed inside (left of the outward normal)
    "ghost_left_depth": ("ora_hllc(g, h_dry, hi, un, ut, value, un, ut, G);",
                         "ora_hllc(g, h_dry, value, un, ut, hi, un, ut, G);"),
    # fixed stage: ghost placed inside
    "ghost_left_stage": ("ora_hllc(g, h_dry, hi, un, ut, hb, un, ut, G);",
                         "ora_hllc(g, h_dry, hb, un, ut, hi, un, ut, G);"),
    # fixed depth: ghost at rest along the edge
    "ghost_zero_tangential": (
        "ora_hllc(g, h_dry, hi, un, ut, value, un, ut, G);",
        "ora_hllc(g, h_dry, hi, un, ut, value, un, 0.0, G);"),
    # monitors: inward instead of outward rate
    "monitor_rate_sign": ("o->brate[e] = -o->cl[3 * e];",
                          "o->brate[e] = o->cl[3 * e];"),
    # monitors: volume summed without the time step
    "monitor_volume_no_dt": ("o->bvol[e] += dt * o->brate[e];",
                             "o->bvol[e] += o->brate[e];"),
    # envelope: wetting time taken at the start of the step
    "wet_time_start": ("o->twet[i] = tn;", "o->twet[i] = o->t;"),
    # envelope: maximum tracked on wet cells only
    "hmax_wet_only": ("if (out[0] > o->hmax[i]) o->hmax[i] = out[0];",
                      "if (out[0] > o->hmax[i] && out[0] > h_dry) "
                      "o->hmax[i] = out[0];"),
}


def _plant(name, workdir):
    old, new = PLANTED[name]
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"{name}: anchor not found exactly once"
    path = os.path.join(workdir, f"{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(workdir, f"lib{name}.so")
    O.compile_to(path, lib)
    env = dict(os.environ, SWE_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                        "-p", "no:cacheprovider", *PINS], cwd=ROOT, env=env,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       timeout=600)
    return name, r.returncode, r.stdout.decode()[-400:]


def test_every_planted_mistake_fails_a_pin():
    work = tempfile.mkdtemp(prefix="swe_planted_")
    try:
        with ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda n: _plant(n, work), PLANTED))
    finally:
        shutil.rmtree(work, ignore_errors=True)
    survived = [(n, out) for n, rc, out in results if rc == 0]
    assert not survived, f"pins missed planted mistakes: {survived}"
    crashed = [(n, rc) for n, rc, _ in results if rc not in (0, 1)]
    assert not crashed, crashed
