"""The oracle's pins have teeth: plausible mistakes planted in a copy of the oracle (on
the CPU, in a temporary build) must each make at least one pin fail."""
import os
import shutil
import tempfile

import pytest

import oracle
import test_oracle_pins as pins

MUTANTS = {
    "h drops alpha": ("*h = S2 + alpha;", "*h = S2;"),
    "g sign flipped": ("*g = *P - S1;", "*g = S1 - *P;"),
    "P drops beta": ("*P = sumA_k + alpha * xk + beta;", "*P = sumA_k + alpha * xk;"),
    "S2 wrong power": ("S2 += v[l] * q * q;", "S2 += v[l] * q;"),
    "derivative wrong column": ("double q = A[(int64_t)idx[l] * r + k] / (Ax[l] + eps_log);",
                                "double q = A[(int64_t)idx[l] * r] / (Ax[l] + eps_log);"),
    "model update sign": ("double m = Ax[l] + d * A[(int64_t)idx[l] * r + k];",
                          "double m = Ax[l] - d * A[(int64_t)idx[l] * r + k];"),
    "Newton sign": ("double xn = x[k] - g / h;", "double xn = x[k] + g / h;"),
    "guard removed": ("if (prm->guard && d < 0.0) {", "if (0) {"),
    "Ax ignores x": ("if (x[k] != 0.0) s += a[k] * x[k];", "if (x[k] != 0.0) s += a[k];"),
    "objective drops -v": ("cj += v * log(v / M) - v;", "cj += v * log(v / M);"),
    "column_kl drops -v": ("kl += v[l] * log(v[l] / M) - v[l];", "kl += v[l] * log(v[l] / M);"),
    "column_kl drops sumA x": ("for (int32_t k = 0; k < r; ++k) kl += sumA[k] * x[k];",
                               "for (int32_t k = 0; k < r; ++k) kl += 0.0 * sumA[k] * x[k];"),
    "objective drops model mass": ("total += sw[k] * sf[k];", "total += sw[k];"),
    "sums wrong column": ("sumA[k] += A[p * r + k];", "sumA[k] += A[p * r];"),
    "philox drops key": ("uint64_t n0 = hi1 ^ c1 ^ k0,", "uint64_t n0 = hi1 ^ c1,"),
    "shuffle bound off by one": ("(((__uint128_t)w * (uint64_t)(i + 1)) >> 64)",
                                 "(((__uint128_t)w * (uint64_t)(i)) >> 64)"),
    "W-half uses F regulariser": ("ids, prm,\n               st, sumF_out);",
                                  "ids, prm,\n               st, sumF_out); (void)0;"),
    "break test inverted": ("(fabs(dN) < prm->eps_x * xs)", "(fabs(dN) > prm->eps_x * xs)"),
    "W-half wrong alpha": ("half_sweep(n, csr_ptr, csr_idx, csr_val, m, F, W, r, prm->alpha_W, prm->beta_W,",
                           "half_sweep(n, csr_ptr, csr_idx, csr_val, m, F, W, r, prm->alpha_F, prm->beta_F,"),
}
# a no-op edit is not a mutant
del MUTANTS["W-half uses F regulariser"]

PIN_TESTS = [
    ("test_philox_block_matches_numpy", dict(ctr=[5, 3, 1, 0], key=[7, 0])),
    ("test_permutation_valid_and_uniform", {}),
    ("test_subproblem_value_matches_library_kl", dict(alpha=1.3, beta=2.1)),
    ("test_derivatives_match_finite_differences", dict(alpha=0.9, beta=0.4)),
    ("test_inner_loop_matches_1d_minimiser", dict(alpha=0.5, beta=0.2)),
    ("test_inner_loop_production_tolerances_never_increase", {}),
    ("test_guard_rejects_overshooting_decrease", {}),
    ("test_objective_matches_dense_library_kl", {}),
    ("test_column_kl_matches_library_kl", {}),
    ("test_factor_sums_match_numpy", {}),
    ("test_half_sweeps_never_increase_objective", {}),
    ("test_r1_closed_form_independence_model", {}),
    ("test_r1_regularised_closed_form", {}),
    ("test_r1_regularised_closed_form_W_half", {}),
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not found exactly once"
    tag = "".join(c if c.isalnum() else "_" for c in name)
    csrc = os.path.join(workdir, f"{tag}.c")
    with open(csrc, "w") as fh:
        fh.write(src.replace(old, new))
    lib = oracle.load(oracle.build(force=True, src=csrc, out=os.path.join(workdir, f"{tag}.so")))
    saved = oracle._lib
    oracle._lib = lib
    caught = []
    try:
        for test, kw in PIN_TESTS:
            try:
                getattr(pins, test)(oracle, **kw)
            except (AssertionError, FloatingPointError, ValueError, IndexError):
                caught.append(test)
                break
    finally:
        oracle._lib = saved
    assert caught, f"no pin caught the mutant {name!r}"
