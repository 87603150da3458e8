"""The oracle's pins catch plausible mistakes.

Each case copies the oracle source, plants one mistake by replacing one line
(a flipped sign, a dropped division, a missing stencil plane, ...), builds the
copy with gcc and the oracle's own flags, and runs the pin tests against it in
a subprocess.  The pins
must fail for every mutant.  Nothing here touches the GPU path.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mech_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_adjoint.py"]

MUTANTS = {
    "adhesion_sign": ("double s = kappa * delta - gamma * sqrt(rho * delta);",
                      "double s = kappa * delta + gamma * sqrt(rho * delta);"),
    "rho_no_division": ("double rho = (ri * rj) / (ri + rj);                  /* combined radius */",
                        "double rho = (ri * rj);                  /* combined radius */"),
    "force_x_sign": ("f[0] += s * ex;", "f[0] -= s * ex;"),
    "diameter_as_radius": ("force_ctx *C = (force_ctx *)c;\n    pair_force(C->kappa, C->gamma, C->x[i], C->y[i], C->z[i], 0.5 * C->d[i],",
                           "force_ctx *C = (force_ctx *)c;\n    pair_force(C->kappa, C->gamma, C->x[i], C->y[i], C->z[i], 1.0 * C->d[i],"),
    "missing_plane": ("    for (int dz = -1; dz <= 1; ++dz) {\n        int64_t cz = iz + dz;",
                      "    for (int dz = -1; dz <= 0; ++dz) {\n        int64_t cz = iz + dz;"),
    "always_clamp": ("    if (vn > m) {\n        double sc = m / vn;",
                     "    if (vn >= 0.0) {\n        double sc = m / vn;"),
    "unstable_placement": ("    for (int64_t i = 0; i < n; ++i) {            /* stable placement */",
                           "    for (int64_t i = n - 1; i >= 0; --i) {            /* stable placement */"),
    "binning_rounds": ("int64_t i = (int64_t)floor((p - o) / e);",
                       "int64_t i = (int64_t)floor((p - o) / e + 0.5);"),
    "adjoint_srho_sign": ("double s_rho = -C->gamma * delta / (2.0 * sq);",
                          "double s_rho = C->gamma * delta / (2.0 * sq);"),
    "adjoint_drop_sdelta": ("C->pb[k] += (s / l) * (w[k] - e[k] * q) - s_delta * q * e[k];",
                            "C->pb[k] += (s / l) * (w[k] - e[k] * q);"),
    # acceptance-test scales: an allowance or scale that is too large must be
    # caught as well as one that is too small
    "tol_drop_onset_guard": ("    if (delta > -eta) {\n        double dm = delta > eta ? delta : eta;",
                             "    if (1) {\n        double dm = delta > eta ? delta : eta;"),
    "tol_eta_x16": ("    double eta = 4.0 * C->u * (ri + rj + l);\n    if (delta > 0.0 && l > 0.0) {",
                    "    double eta = 64.0 * C->u * (ri + rj + l);\n    if (delta > 0.0 && l > 0.0) {"),
    "tol_S_sign": ("C->S += C->kappa * delta + C->gamma * sqrt(rho * delta);",
                   "C->S += C->kappa * delta - C->gamma * sqrt(rho * delta);"),
    "adjtol_drop_fj": ("double W = fi + fj;", "double W = fi;"),
    "adjtol_drop_sdelta": ("C->Sp += W * (2.0 * fabs(s) / l + fabs(s_delta));",
                           "C->Sp += W * (2.0 * fabs(s) / l);"),
    "adjtol_eta_x16": ("    const double eta = 4.0 * C->u * (ri + rj + l);",
                       "    const double eta = 64.0 * C->u * (ri + rj + l);"),
    "adjoint_clamp_projection": ("for (int k = 0; k < 3; ++k) o[k] = sc * (g[k] - vh[k] * vg);",
                                 "for (int k = 0; k < 3; ++k) o[k] = sc * g[k];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    import oracle
    subprocess.run(["gcc", *oracle._CFLAGS, "-o", str(lib), str(mutant_c), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "Error" in r.stdout
