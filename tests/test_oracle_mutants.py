"""Planted mistakes: each mutant copies the oracle's C source, changes one
thing a careless implementation could get wrong, builds it on the CPU and
runs the whole pin battery in a child process.  Some pin must fail for every
mutant; a mutant that passes every pin would mean the pins cannot tell that
mistake from the right arithmetic."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, text in ccg_oracle.c, replacement, expected number of occurrences;
# a count above one plants the same mistake in every copy of the line)
MUTANTS = [
    ("beta_drops_alpha_over_omega",
     "zc beta = zdiv(rho, rho_old) * zdiv(alpha, omega);",
     "zc beta = zdiv(rho, rho_old);", 3),
    ("omega_conjugated",
     "omega = CMPLX(creal(ts) / tt, cimag(ts) / tt);",
     "omega = CMPLX(creal(ts) / tt, -cimag(ts) / tt);", 3),
    ("p_update_sign",
     "p[i] = r[i] + beta * (p[i] - omega * v[i]);",
     "p[i] = r[i] + beta * (p[i] + omega * v[i]);", 2),
    ("s_update_sign",
     "s[i] = r[i] - alpha * v[i];", "s[i] = r[i] + alpha * v[i];", 2),
    ("adjoint_without_conj",
     "y[j] += conj(A[i * lda + j]) * xi;", "y[j] += A[i * lda + j] * xi;", 1),
    ("cgnr_beta_inverted",
     "double beta = gamma_new / gamma;", "double beta = gamma / gamma_new;", 1),
    ("matvec_transposed",
     "s += A[i * lda + j] * x[j];\n        y[i] = s;\n    }\n}\n\n/* y = A^H x",
     "s += A[j * lda + i] * x[j];\n        y[i] = s;\n    }\n}\n\n/* y = A^H x", 1),
    ("dot_unconjugated",
     "s += conj(a[i]) * b[i];", "s += a[i] * b[i];", 1),
    ("stop_test_not_squared",
     "const double thr2 = tol * tol * ny2;", "const double thr2 = tol * ny2;", 7),
    ("residual_sign",
     "rt[i] = y[i] - rt[i];", "rt[i] = y[i] + rt[i];", 1),
    ("division_without_conj",
     "zc q = a * conj(b);", "zc q = a * b;", 1),
    ("x_update_drops_omega_s",
     "x[i] = x[i] + alpha * p[i] + omega * s[i];", "x[i] = x[i] + alpha * p[i];",
     2),
    ("r_update_wrong_vector",
     "r[i] = s[i] - omega * t[i];", "r[i] = s[i] - omega * s[i];", 2),
    ("cgnr_p_update_drops_beta",
     "p[i] = z[i] + beta * p[i];", "p[i] = z[i];", 1),
    ("rho_without_shadow",
     "rho = dotc(n, rh, r);", "rho = dotc(n, r, r);", 2),
    ("sigma_without_shadow",
     "zc sigma = dotc(n, rh, v);", "zc sigma = dotc(n, r, v);", 2),
    ("ts_operands_swapped",
     "zc ts = dotc(n, t, s);", "zc ts = dotc(n, s, t);", 2),
    ("norm_drops_imaginary",
     "s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);",
     "s += creal(v[i]) * creal(v[i]);", 1),
    ("cgnr_alpha_halved",
     "double alpha = gamma / ww;", "double alpha = 0.5 * gamma / ww;", 1),
    ("half_step_forgets_x",
     "x[i] = x[i] + alpha * p[i];\n            k++;",
     "(void)p;\n            k++;", 1),
    ("cgnr_r_update_sign",
     "r[i] = r[i] - alpha * w[i];\n        }\n        rr = norm2sq(n, r);\n        k++;\n        if (!isfinite(rr)) {\n            st->info = 4;\n            break;\n        }\n        if (hist) {\n            hist[k - 1].alpha_re = alpha;",
     "r[i] = r[i] + alpha * w[i];\n        }\n        rr = norm2sq(n, r);\n        k++;\n        if (!isfinite(rr)) {\n            st->info = 4;\n            break;\n        }\n        if (hist) {\n            hist[k - 1].alpha_re = alpha;",
     1),
    ("cocg_pq_conjugated",
     "zc pq = dotu(n, p, q);", "zc pq = dotc(n, p, q);", 1),
    ("cocg_alpha_conj",
     "zc alpha = zdiv(rho, pq);", "zc alpha = zdiv(rho, conj(pq));", 1),
    ("cocr_ww_conjugated",
     "zc ww = dotu(n, w, w);", "zc ww = dotc(n, w, w);", 1),
    ("cocr_w_update_drops_beta",
     "w[i] = u[i] + beta * w[i];", "w[i] = u[i];", 1),
    ("cocr_alpha_inverted",
     "zc alpha = zdiv(rho, ww);", "zc alpha = zdiv(ww, rho);", 1),
    ("bilinear_form_conjugated",
     "s += a[i] * b[i];", "s += conj(a[i]) * b[i];", 1),
    ("mixed_update_unscaled",
     "x[i] = x[i] + nr * (zc)d32[i];", "x[i] = x[i] + (zc)d32[i];", 1),
    ("mixed_residual_not_normalised",
     "const double scale = 1.0 / nr;", "const double scale = 1.0;", 2),
    ("c64_product_transposed",
     "s += A[i * lda + j] * x[j];\n        y[i] = s;\n    }\n}\n\nstatic double norm2sq_c64",
     "s += A[j * lda + i] * x[j];\n        y[i] = s;\n    }\n}\n\nstatic double norm2sq_c64", 1),
    ("cocr_r_update_wrong_vector",
     "r[i] = r[i] - alpha * w[i];\n        }\n        rr = norm2sq(n, r);\n        k++;\n        if (!isfinite(rr)) {\n            st->info = 4;\n            break;\n        }\n        if (hist) {\n            hist[k - 1].alpha_re = creal(alpha);",
     "r[i] = r[i] - alpha * u[i];\n        }\n        rr = norm2sq(n, r);\n        k++;\n        if (!isfinite(rr)) {\n            st->info = 4;\n            break;\n        }\n        if (hist) {\n            hist[k - 1].alpha_re = creal(alpha);",
     1),
    ("sym_lower_read_from_row",
     "s += A[j * lda + i] * x[j];", "s += A[i * lda + j] * x[j];", 1),
    ("sym_diagonal_dropped",
     "for (int64_t j = i; j < n; ++j)\n            s += A[i * lda + j] * x[j];",
     "for (int64_t j = i + 1; j < n; ++j)\n            s += A[i * lda + j] * x[j];", 1),
    ("wide_product_transposed",
     "s += A[i * lda + j] * (fc)x[j];", "s += A[j * lda + i] * (fc)x[j];", 1),
    ("wide_update_unscaled",
     "x[i] = x[i] + CMPLX(nr * creal(d[i]), nr * cimag(d[i]));", "x[i] = x[i] + d[i];", 1),
    ("wide_rhs_not_normalised",
     "b[i] = CMPLX(creal(r[i]) * scale, cimag(r[i]) * scale);", "b[i] = r[i];", 1),
    ("inner_breakdown_ignored",
     "if ((info_in == 2 || info_in == 3) && it == 0) {", "if (0) {", 2),
]


@pytest.mark.parametrize("name,old,new,count", MUTANTS,
                         ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new, count):
    src = open(oracle.SRC).read()
    assert src.count(old) == count, "mutation site moved: %s" % name
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = oracle.build(str(mutated), str(tmp_path / "libmutant.so"))
    proc = subprocess.run([sys.executable, os.path.join(HERE, "mutant_runner.py"),
                           lib], capture_output=True, text=True, timeout=300)
    failed = [ln for ln in proc.stdout.splitlines() if ln.startswith("FAILED")]
    crashed = proc.returncode != 0
    assert failed or crashed, "no pin caught mutant %s" % name


def test_pins_pass_on_unmutated_copy(tmp_path):
    lib = oracle.build(oracle.SRC, str(tmp_path / "libcopy.so"))
    proc = subprocess.run([sys.executable, os.path.join(HERE, "mutant_runner.py"),
                           lib], capture_output=True, text=True, timeout=300)
    assert proc.returncode == 0, proc.stderr
    assert "FAILED" not in proc.stdout, proc.stdout
