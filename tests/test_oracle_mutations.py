"""The oracle's pins catch planted mistakes.

Each case copies the oracle source, plants one plausible mistake (a dropped
term, a wrong sign, a wrong index or scale), builds it into a temporary
library and runs the pin suite against it in a child process: the suite must
fail.  Mistakes are planted in the oracle, on the CPU, never in GPU code.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle_en.c")

MUTATIONS = {
    "prox_scale": ("if (t > thr) return (t - thr) / den;", "if (t > thr) return (t - thr) / (1.0 + l2);"),
    "pstar_factor": ("return s / (2.0 * l2);", "return s / l2;"),
    "grad_sign_b": ("g[i] = y[i] + b[i] - Au[i];", "g[i] = y[i] - b[i] - Au[i];"),
    "grad_psi_sign": ("g[i] = y[i] + b[i] - u[i];", "g[i] = y[i] + b[i] + u[i];"),
    "tie_active": ("if (t > thr) { J[r]", "if (t >= thr) { J[r]"),
    "newton_identity": ("double v = kappa * s + (i == l ? 1.0 : 0.0);", "double v = kappa * s;"),
    "chol_sign": ("for (int64_t k = 0; k < j; ++k) t -= V[i * m + k] * V[j * m + k];",
                  "for (int64_t k = 0; k < j; ++k) t += V[i * m + k] * V[j * m + k];"),
    "ls_second_order": ("ei = 0.5 * s * s * kappa * wd[i] * wd[i];", "ei = 0.5 * s * kappa * wd[i] * wd[i];"),
    "eta_sign": ("double p = orc_prox_sp(x[j] - g[j], 1.0, l1, l2);", "double p = orc_prox_sp(x[j] + g[j], 1.0, l1, l2);"),
    "dual_sign": ("return -hs - ps;", "return -hs + ps;"),
    "multiplier_update": ("x[i] = u[i];           /* x - sigma(A^T y + z) */",
                          "x[i] = t[i];           /* x - sigma(A^T y + z) */"),
    "gemv_index": ("for (int64_t i = 0; i < m; ++i) s += a[i] * v[i];", "for (int64_t i = 1; i < m; ++i) s += a[i] * v[i];"),
    "psi_l2_term": ("return 0.5 * dot(y, y, m) + dot(b, y, m) + (1.0 + sigma * l2) / (2.0 * sigma) * pp -",
                    "return 0.5 * dot(y, y, m) + dot(b, y, m) + 1.0 / (2.0 * sigma) * pp -"),
    "conj_prox": ("if (v >= thr) return (v * l2 + l1) / den;", "if (v >= thr) return (v * l2 - l1) / den;"),
    "df_ridge": ("for (int64_t p = 0; p < r; ++p) M[p * r + p] += lambda2;",
                 "for (int64_t p = 0; p < r; ++p) M[p * r + p] += 2.0 * lambda2;"),
    "gcv_square": ("gcv = (rss / md) / ((1.0 - nu / md) * (1.0 - nu / md));", "gcv = (rss / md) / (1.0 - nu / md);"),
    "ebic_log_n": ("ebic = log(rss / md) + (nu / md) * (log(md) + log((double)n));",
                   "ebic = log(rss / md) + (nu / md) * log(md);"),
    "lasso_theta": ("if (amax > l1) theta = l1 / amax;", "if (amax > l1) theta = 1.0;"),
    "cv_validation_rows": ("if (fold[i] == f) s += (res[i] - b[i]) * (res[i] - b[i]);",
                           "if (fold[i] != f) s += (res[i] - b[i]) * (res[i] - b[i]);"),
    "cg_beta": ("const double beta = rr_new / rr;", "const double beta = rr / rr_new;"),
    "cg_matvec_kappa": ("for (int64_t i = 0; i < m; ++i) q[i] = p[i] + kappa * q[i];",
                        "for (int64_t i = 0; i < m; ++i) q[i] = p[i] + q[i];"),
    "cg_stop_square": ("const double stop = eps * eps * dot(g, g, m);", "const double stop = eps * dot(g, g, m);"),
    "cg_residual": ("      res[i] -= alpha * q[i];", "      res[i] -= alpha * p[i];"),
    "cg_steepest": ("for (int64_t i = 0; i < m; ++i) p[i] = res[i] + beta * p[i];",
                    "for (int64_t i = 0; i < m; ++i) p[i] = res[i] + 0.0 * beta * p[i];"),
    "debias_rhs": ("for (int64_t i = 0; i < m; ++i) s += A[J[p] * lda + i] * b[i];",
                   "for (int64_t i = 1; i < m; ++i) s += A[J[p] * lda + i] * b[i];"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    (tmp_path / "oracle_en.h").write_text(open(os.path.join(ROOT, "oracle", "oracle_en.h")).read())
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-I", str(tmp_path), "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, SSNAL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} was not caught by any pin:\n{r.stdout[-2000:]}"
