"""The oracle's pins must be strong enough to catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source (a
dropped term, a wrong sign or index, the weight inside the root, ...), builds it
into a temporary library, and runs the pin suite against it: at least one pin
must fail. Nothing here touches the GPU library.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pwbf_oracle.c")

MUTANTS = {
    "first_fire_max": ("if (v < first) first = v;", "if (v > first) first = v;"),
    "drop_cos_theta": ("double t_tx = (x * sin(th) + z * cos(th) - first) / g->c;",
                       "double t_tx = (x * sin(th) + z - first) / g->c;"),
    "steer_sign": ("double t_tx = (x * sin(th) + z * cos(th) - first) / g->c;",
                   "double t_tx = (-x * sin(th) + z * cos(th) - first) / g->c;"),
    "rx_index_sign": ("double dxe = x - g->elem_x[e];", "double dxe = x + g->elem_x[e];"),
    "aperture_width": ("double half_aperture = z / (2.0 * g->f_number);",
                       "double half_aperture = z / (g->f_number);"),
    "interp_off_by_one": ("if (n0 >= 0.0 && n0 < (double)ns) a = u[(int64_t)n0];",
                          "if (n0 >= 1.0 && n0 < (double)ns) a = u[(int64_t)n0 - 1];"),
    "clamp_not_zero": ("if (n0 + 1.0 >= 0.0 && n0 + 1.0 < (double)ns) b = u[(int64_t)n0 + 1];",
                       "b = u[(int64_t)(n0 + 1.0 < ns ? (n0 + 1.0 < 0 ? 0 : n0 + 1.0) : ns - 1)];"),
    "t0_sign": ("return (t_tx + t_rx - g->t0[a]) * g->fs;",
                "return (t_tx + t_rx + g->t0[a]) * g->fs;"),
    "weight_inside_root": ("s[e] = ora_apod_weight(g, e, x, z) * sgn(v) * sqrt(fabs(v));",
                           "s[e] = sgn(v) * sqrt(fabs(ora_apod_weight(g, e, x, z) * v));"),
    "pixel_axes_swapped": ("int64_t ix = p / g->nz, iz = p % g->nz;",
                           "int64_t iz = p / g->nx, ix = p % g->nx;"),
    "dmas_not_halved": ("return 0.5 * (sum * sum - sq);", "return (sum * sum - sq);"),
    "hann_half_period": ("return 0.5 * (1.0 + cos(M_PI * d / half_aperture));",
                         "return 0.5 * (1.0 + cos(0.5 * M_PI * d / half_aperture));"),
    "pdas_power_inside": ("yt += ora_apod_weight(g, e, x, z) * sgn(v) * pow(fabs(v), 1.0 / p);",
                          "yt += ora_apod_weight(g, e, x, z) * sgn(v) * pow(fabs(v), p);"),
    "pdas_weight_inside_root": (
        "yt += ora_apod_weight(g, e, x, z) * sgn(v) * pow(fabs(v), 1.0 / p);",
        "yt += sgn(v) * pow(fabs(ora_apod_weight(g, e, x, z) * v), 1.0 / p);"),
    "pdas_unsigned_power": ("return sgn(yt) * pow(fabs(yt), p);", "return pow(fabs(yt), p);"),
    "pdas_root_order": ("return sgn(yt) * pow(fabs(yt), p);",
                        "return sgn(yt) * pow(fabs(yt), 1.0 / p);"),
    "iq_rotation_sign": ("const double ph = 2.0 * M_PI * fd * s / g->fs;",
                         "const double ph = -2.0 * M_PI * fd * s / g->fs;"),
    "iq_no_rotation": ("const double ph = 2.0 * M_PI * fd * s / g->fs;",
                       "const double ph = 0.0 * fd * s;"),
    "bbdmas_no_root": ("const double k = amp > 0.0 ? 1.0 / sqrt(amp) : 0.0;",
                       "const double k = 1.0;"),
    "bbdmas_weight_inside_root": ("    sr += w * vr;\n    si += w * vi;",
                                  "    sr += (form == 1 ? sqrt(w) : w) * vr;\n"
                                  "    si += (form == 1 ? sqrt(w) : w) * vi;"),
    "bbdmas_not_squared": ("    *yr = sr * sr - si * si;\n    *yi = 2.0 * sr * si;",
                           "    *yr = sr;\n    *yi = si;"),
    "compound_keeps_last": (
        "for (int32_t a = 0; a < g->n_angles; ++a) y += das_one_angle(g, rf, a, first[a], x, z);",
        "for (int32_t a = 0; a < g->n_angles; ++a) y = das_one_angle(g, rf, a, first[a], x, z);"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation anchor drifted from the oracle source"
    msrc = tmp_path / "pwbf_oracle.c"
    msrc.write_text(src.replace(old, new))
    mlib = tmp_path / "liboracle.so"
    mlib_omp = tmp_path / "liboracle_omp.so"
    for lib, extra in ((mlib, []), (mlib_omp, ["-fopenmp"])):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                               *extra, "-o", str(lib), str(msrc), "-lm"])
    code = (f"import oracle; oracle._LIB={str(mlib)!r}; oracle._LIB_OMP={str(mlib_omp)!r}; "
            f"oracle._SRC={str(msrc)!r}; "
            "import sys, pytest; sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', "
            f"{os.path.join(ROOT, 'tests', 'test_oracle_pins.py')!r}]))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 1, f"no pin failed for mutant {name}:\n{r.stdout[-2000:]}"
