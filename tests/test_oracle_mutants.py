"""Plants plausible mistakes in copies of the oracle (on the CPU) and checks that the pins in
test_oracle_pins.py catch every one of them."""
import os
import shutil
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "oracle.h")

# (name, original text, mutated text): every original occurs exactly once in oracle.c
MUTANTS = [
    ("drop lambda", "double t = vals[i] * (lambda ? lambda[j] : 1.0);", "double t = vals[i];"),
    ("include own mode", "if (m != n) t *= A[m][(int64_t)l[m] * R + j];",
     "t *= A[m][(int64_t)l[m] * R + j];"),
    ("transposed factor", "if (m != n) t *= A[m][(int64_t)l[m] * R + j];",
     "if (m != n) t *= A[m][(int64_t)j * dims[m] + l[m]];"),
    ("model drops lambda", "double t = lambda ? lambda[j] : 1.0;", "double t = 1.0;"),
    ("forward sign", "for (int q = 0; q < c; ++q) s -= L[c * R + q] * y[q];",
     "for (int q = 0; q < c; ++q) s += L[c * R + q] * y[q];"),
    ("cholesky transposed", "for (int k = 0; k < c; ++k) s -= L[r * R + k] * L[c * R + k];",
     "for (int k = 0; k < c; ++k) s -= L[r * R + k] * L[k * R + c];"),
    ("hadamard includes own gram", "        if (m != n)\n            for (int a = 0; a < R * R; ++a) Gam[a]",
     "        if (1)\n            for (int a = 0; a < R * R; ++a) Gam[a]"),
    ("norm not square-rooted", "lambda[j] = sqrt(s);", "lambda[j] = s;"),
    ("fit cross term", "double r2 = xx - 2.0 * xm + mm;", "double r2 = xx - xm + mm;"),
    ("gcp derivative sign", "case 0: return exp(m) - x;", "case 0: return exp(m) + x;"),
    ("logit derivative", "case 1: return 1.0 / (1.0 + exp(-m)) - x;", "case 1: return 1.0 / (1.0 + exp(m)) - x;"),
    ("gaussian derivative factor", "default: return 2.0 * (m - x);", "default: return (m - x);"),
    ("gaussian loss sign", "default: return (x - m) * (x - m);", "default: return (x + m) * (x - m);"),
    ("gamma derivative sign", "case 3: return 1.0 / (m + ORACLE_GAMMA_EPS) - x /",
     "case 3: return 1.0 / (m + ORACLE_GAMMA_EPS) + x /"),
    ("gamma loss log term", "+ log(m + ORACLE_GAMMA_EPS);", "- log(m + ORACLE_GAMMA_EPS);"),
    ("philox key bump", "k1 += 0xBB67AE8584CAA73Bull;", "k1 += 0x9E3779B97F4A7C15ull;"),
    ("zero-sample weight", "(cells - (double)P) / (double)s_z", "cells / (double)s_z"),
    ("adam bias correction", "const double mh = m[i] / c1,", "const double mh = m[i],"),
    ("unstable perm", "for (int64_t i = 0; i < P; ++i) {\n        int32_t k = subs[i * d + n];",
     "for (int64_t i = P - 1; i >= 0; --i) {\n        int32_t k = subs[i * d + n];"),
    ("bf16 ties away", "? hi_bits : lo_bits; /* tie", "? lo_bits : hi_bits; /* tie"),
    ("bf16 f64 rounds twice", "const double a = fabs(v);", "const double a = (double)(float)fabs(v);"),
    ("bf16 f64 no subnormal step", "const int qe = (e - 8 < -133) ? -133 : e - 8;",
     "const int qe = e - 8;"),
    ("bf16 f64 ties odd", "pick = (fmod(k, 2.0) == 0.0) ? lo : hi;", "pick = (fmod(k, 2.0) == 0.0) ? hi : lo;"),
]

CHECKS = [
    (pins.test_mttkrp_brute_force, dict(dims=(4, 5, 6), R=3)),
    (pins.test_mttkrp_brute_force, dict(dims=(3, 2, 5, 4), R=7)),
    (pins.test_mttkrp_rank1_closed_form, {}),
    (pins.test_mttkrp_two_way_is_sparse_matrix_product, {}),
    (pins.test_perm_matches_stable_argsort, dict(I=17)),
    (pins.test_model_values_and_gram_match_dense, {}),
    (pins.test_fit_matches_brute_force_residual, {}),
    (pins.test_cp_als_mode_solves_normal_equations_and_matches_lstsq, {}),
    (pins.test_gcp_poisson_loss_dense_and_gradient_finite_differences, {}),
    (pins.test_gcp_losses_dense_and_finite_differences, dict(loss="bernoulli")),
    (pins.test_gcp_losses_dense_and_finite_differences, dict(loss="gaussian")),
    (pins.test_gcp_losses_dense_and_finite_differences, dict(loss="gamma")),
    (pins.test_bf16_rne_matches_torch_on_samples_and_boundaries, {}),
    (pins.test_bf16_rne_f64_matches_exact_rounding_and_fp32_rounding, {}),
    (pins.test_philox_matches_numpy_philox, {}),
    (pins.test_gcp_sample_is_unbiased_and_uniform, {}),
    (pins.test_adam_constant_gradient_closed_form, {}),
]


def test_unmutated_oracle_passes_checks():
    for fn, kw in CHECKS:
        fn(**kw)


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, orig, mut):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation site for '{name}' not unique"
    (tmp_path / "oracle.c").write_text(src.replace(orig, mut))
    shutil.copy(HDR, tmp_path / "oracle.h")
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-w",
                    "-o", str(lib), str(tmp_path / "oracle.c"), "-lm"], check=True)
    prev = oracle._swap_library(str(lib))
    caught = []
    try:
        for fn, kw in CHECKS:
            try:
                fn(**kw)
            except (AssertionError, oracle.OracleError) as e:
                caught.append((fn.__name__, type(e).__name__))
                break
    finally:
        oracle._restore_library(prev)
    assert caught, f"mutant '{name}' survived every pin"
