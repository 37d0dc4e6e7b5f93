"""Planted mistakes in a copy of the oracle must fail its pins.

A pin is only worth something if a plausible slip in the oracle breaks it. Each case below
copies the oracle package into a temporary directory, makes one such slip there (a wrong
index or operand, a dropped factor, term or sign, a swapped parity, an inverted ratio),
builds the copy's C library and runs, in a fresh interpreter that imports the copy, the
pin tests meant to catch that slip. The case passes when at least one of them fails. The
unchanged oracle passes every pin (the rest of this suite), so a failure here is caused by
the slip alone.

CPU only: nothing here loads the GPU library, and the slips live in the temporary copy.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PINS = "tests/test_oracle_pins.py::"
SOURCE = "tests/test_oracle_source.py"
FUNCTIONAL = "tests/test_oracle_functional.py"
PROPOSAL = "tests/test_oracle_proposal.py::"
LEVEL_MEANS = PINS + "test_level_means_match_dense_strang_products"
BIAS = PINS + "test_bias_estimate_bounds_the_true_splitting_bias"
DRIVER_LEVELS = PINS + "test_adaptive_driver_adds_the_levels_the_bias_requires"
C = "mlmc_oracle.c"

# (name, file in oracle/, [(text, replacement)], pin tests that must catch it)
PLANTS = [
    # Philox4x32-10 (Salmon et al., SC'11)
    ("philox wrong multiplier operand", C,
     [("uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;",
       "uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x1;")],
     [PINS + "test_philox_matches_rocrand"]),
    ("philox same Weyl increment for both key words", C,
     [("k1 += 0xBB67AE85u;", "k1 += 0x9E3779B9u;")],
     [PINS + "test_philox_matches_rocrand"]),
    # logarithm of the exponential holding times
    ("log without the tail of ln 2", C,
     [("return de * ln2_head + (de * ln2_tail + b);", "return de * ln2_head + b;")],
     [PINS + "test_log_within_two_ulp_on_the_uniform_grid"]),
    ("log series coefficient 1/6 for 1/5", C,
     [("p = fma(p, z, 1.0 / 5.0);", "p = fma(p, z, 1.0 / 6.0);")],
     [PINS + "test_log_within_two_ulp_on_the_uniform_grid"]),
    # decomposition A = D - T (section 2.1)
    ("d without r", C,
     [("d[i] = diag + ri;", "d[i] = diag;")],
     [PINS + "test_decomposition_identity_and_fields"]),
    ("sign of the positive entries", C,
     [("slot_sign[s + k] = (uint8_t)(val[e] < 0.0);", "slot_sign[s + k] = (uint8_t)(val[e] > 0.0);")],
     [PINS + "test_decomposition_identity_and_fields"]),
    # alias tables of the jump law
    ("alias leftover without the unit", C,
     [("slot_alias[s + a] = g;\n            q[g] = (q[g] + q[a]) - 1.0;",
       "slot_alias[s + a] = g;\n            q[g] = q[g] - q[a];")],
     [PINS + "test_alias_tables_reproduce_the_jump_law"]),
    ("alias threshold complemented", C,
     [("slot_thr[s + a] = (uint32_t)floor(q[a] * 4294967296.0);",
       "slot_thr[s + a] = (uint32_t)floor((1.0 - q[a]) * 4294967296.0);")],
     [PINS + "test_alias_tables_reproduce_the_jump_law"]),
    # Algorithm 2
    ("holding time at the old state's rate", C,
     [("double S = -orc_log(orc_uniform(w[2])) * t->inv_r[s];",
       "double S = -orc_log(orc_uniform(w[2])) * t->inv_r[k];")],
     [PINS + "test_one_step_law_matches_the_ctmc_transition_matrix", LEVEL_MEANS]),
    ("coarse functional keeps its sign at a negative jump", C,
     [("o->eta_coarse = phi * coarse;", "o->eta_coarse = coarse;")],
     [LEVEL_MEANS]),
    ("coarse half steps on the wrong parity", C,
     [("const int pair_ends = (n % 2 == 0);", "const int pair_ends = (n % 2 != 0);")],
     [LEVEL_MEANS]),
    ("fine functional loses its closing half step", C,
     [("        fine = fine * exp(t->d[s] * dt / 2.0);\n", "")],
     [LEVEL_MEANS, PINS + "test_diagonal_matrix_is_exact"]),
    ("time step beta / 2N", C,
     [("const double dt = ldexp(beta, -level);", "const double dt = ldexp(beta, -level - 1);")],
     [LEVEL_MEANS, PINS + "test_diagonal_matrix_is_exact"]),
    ("coarse functional not subtracted above l0", C,
     [("y = uj * (o.eta_fine - o.eta_coarse);", "y = uj * o.eta_fine;")],
     [LEVEL_MEANS]),
    # Algorithm 3 (section 5)
    ("source term read at the start row", C,
     [("add_source_point(simpson_weight(n, N), phi * fine, F[s], &integ2, &imag2);",
       "add_source_point(simpson_weight(n, N), phi * fine, F[row], &integ2, &imag2);")],
     [SOURCE]),
    ("coarse source sum with fine weights", C,
     [("add_source_point(simpson_weight(n / 2, N / 2), phi * coarse,",
       "add_source_point(simpson_weight(n, N) / 2.0, phi * coarse,")],
     [SOURCE]),
    ("source sum without grid point 0", C,
     [("add_source_point(simpson_weight(0, N), 1.0, F[s], &integ2, &imag2);", "")],
     [SOURCE]),
    ("Simpson factor 1/2 for 1/3", C,
     [("o->integ_fine = dt / 3.0 * integ2;", "o->integ_fine = dt / 2.0 * integ2;")],
     [SOURCE]),
    ("coarse source terms at odd points too", C,
     [("if (pair_ends) add_source_point(simpson_weight(n / 2", "if (1) add_source_point(simpson_weight(n / 2")],
     [SOURCE]),
    # the forward representation as a scalar functional
    ("start sign dropped", C,
     [("        if (start_neg[l]) y = -y;\n        orc_add(&a1, y);", "        orc_add(&a1, y);")],
     [FUNCTIONAL]),
    ("start rows uniform", C,
     [("uint32_t l = (out[1] < start_thr[slot]) ? slot : (uint32_t)start_alias[slot];\n"
       "        orc_walk_out o;\n"
       "        orc_one_walk(&t, beta, level, key, instance, (int64_t)l, walk, NULL, &o);\n"
       "        double y = w[",
       "uint32_t l = slot;\n"
       "        orc_walk_out o;\n"
       "        orc_one_walk(&t, beta, level, key, instance, (int64_t)l, walk, NULL, &o);\n"
       "        double y = w[")],
     [FUNCTIONAL]),
    ("functional without the coarse term", C,
     [("double y = w[o.final_state] * ((level > l0) ? (o.eta_fine - o.eta_coarse) : o.eta_fine);",
       "double y = w[o.final_state] * o.eta_fine;")],
     [FUNCTIONAL]),
    ("forward deposit at the start row", C,
     [("        const int64_t j = o.final_state;\n", "        const int64_t j = (int64_t)l;\n")],
     [FUNCTIONAL + "::test_forward_deposits_give_every_functional",
      FUNCTIONAL + "::test_forward_level_means_match_dense_strang_products"]),
    ("forward deposit without the start sign", C,
     [("        if (start_neg[l]) y = -y;\n        orc_add(&a1[j], y);",
       "        orc_add(&a1[j], y);")],
     [FUNCTIONAL + "::test_forward_deposits_give_every_functional",
      FUNCTIONAL + "::test_forward_level_means_match_dense_strang_products"]),
    # Algorithm 1's sample sizes and error test
    ("optimal M without the factor 2", "mlmc.py",
     [("np.ceil(2.0 * eps ** -2 *", "np.ceil(eps ** -2 *")],
     [PINS + "test_optimal_sample_sizes_meet_the_variance_budget"]),
    ("bias divided by 2^alpha + 1", "mlmc.py",
     [("/ (2.0 ** ALPHA - 1.0)", "/ (2.0 ** ALPHA + 1.0)")],
     [BIAS, DRIVER_LEVELS]),
    ("bias without the coarser level's term", "mlmc.py",
     [("max(abs(mL), abs(mLm1) / 2.0 ** ALPHA)", "abs(mL)")],
     [BIAS, DRIVER_LEVELS]),
    ("bias with weak order 1", "mlmc.py",
     [("ALPHA = 2.0 ", "ALPHA = 1.0 ")],
     [BIAS, DRIVER_LEVELS]),
    ("per-walk variance without the factor M / (M - 1)", "mlmc.py",
     [("return raw * (M / (M - 1.0)) if M > 1 else raw", "return raw")],
     [PINS + "test_level_variance_is_unbiased_from_two_walks_per_row"]),
    ("level term's root mean square keeps the sampling noise", "mlmc.py",
     [("float(np.mean(m * m)) - level_variance(s1, s2, M) / M", "float(np.mean(m * m))")],
     [PINS + "test_level_term_rms_removes_the_sampling_noise",
      PINS + "test_adaptive_driver_with_a_two_walk_pilot_adds_no_needless_level"]),
    ("driver never adds a level", "mlmc.py",
     [("        L += 1\n        run(L, pilot)", "        break")],
     [BIAS, DRIVER_LEVELS]),
    # the learned proposal
    ("likelihood ratio q/p", "proposal.py",
     [("ratio = np.where(q_slot > 0, p_slot / np.where(q_slot > 0, q_slot, 1.0), 1.0)",
       "ratio = np.where(q_slot > 0, q_slot / p_slot, 1.0)")],
     [PROPOSAL + "test_importance_sampled_levels_are_unbiased"]),
    ("mixing-weight gradient with the wrong sign", "proposal.py",
     [("da = coef * (soft[rows, slot] - p6[rows, slot])", "da = coef * (p6[rows, slot] - soft[rows, slot])")],
     [PROPOSAL + "test_gradients_match_finite_differences"]),
    ("shrinkage gradient without the factor 2", "proposal.py",
     [("2.0 * shrink * (w / W)[:, None]", "shrink * (w / W)[:, None]")],
     [PROPOSAL + "test_gradients_match_finite_differences"]),
]

# A comment-only change, run against the union of the pins above (minus the rocRAND
# cross-check, which needs hipcc).
CONTROL = ("comment only", C,
           [("Decomposition A = D - T (section 2.1).", "Decomposition A = D - T, section 2.1. ")],
           sorted({t for p in PLANTS for t in p[3] if "rocrand" not in t}))

# Runs the named pin tests against the copy at argv[1]: the copy is imported first, so the
# tests' own "from oracle import ..." finds it in sys.modules.
DRIVER = r"""
import sys
copy, root, targets = sys.argv[1], sys.argv[2], sys.argv[3:]
sys.path.insert(0, root)
sys.path.insert(0, copy)
import oracle, oracle.build, oracle.mlmc, oracle.reference, oracle.proposal
assert oracle.__file__.startswith(copy), oracle.__file__
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "-m", "not gpu", "--rootdir", root]
                     + [root + "/" + t for t in targets]))
"""


def _run_plant(base, name, fname, edits, targets):
    """Apply one plant to a fresh copy under `base`, build it and run its pins.
    Returns (pytest exit status, the tail of its output) or an error string."""
    copy = os.path.join(base, "oracle")
    shutil.copytree(os.path.join(ROOT, "oracle"), copy,
                    ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.tmp"))
    path = os.path.join(copy, fname)
    with open(path) as f:
        src = f.read()
    for old, new in edits:
        if src.count(old) != 1:
            return f"the text to change is not found once in oracle/{fname}"
        src = src.replace(old, new)
    with open(path, "w") as f:
        f.write(src)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    b = subprocess.run([sys.executable, os.path.join(copy, "build.py")], env=env,
                       capture_output=True, text=True, timeout=120)
    if b.returncode != 0:
        return "the planted copy does not build:\n" + b.stderr[-2000:]
    r = subprocess.run([sys.executable, "-c", DRIVER, base, ROOT, *targets], cwd=base, env=env,
                       capture_output=True, text=True, timeout=300)
    return r.returncode, "\n".join((r.stdout + r.stderr).splitlines()[-15:])


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """All plants, run side by side (each in its own copy and interpreter)."""
    from tests.native import build_native
    have_rocrand = build_native.rocrand_ref() is not None
    jobs = {}
    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(6, os.cpu_count() or 1))) as ex:
        for k, (name, fname, edits, targets) in enumerate(PLANTS):
            if any("rocrand" in t for t in targets) and not have_rocrand:
                continue
            base = str(tmp_path_factory.mktemp(f"plant{k}"))
            jobs[name] = ex.submit(_run_plant, base, name, fname, edits, targets)
        base = str(tmp_path_factory.mktemp("control"))
        jobs[CONTROL[0]] = ex.submit(_run_plant, base, *CONTROL)
        return {name: job.result() for name, job in jobs.items()}


@pytest.mark.slow
def test_unplanted_copy_passes_the_same_pins(outcomes):
    """Control: a copy changed only in a comment passes every pin the plants use, so the
    failures above come from the plants and not from running against a copy."""
    out = outcomes[CONTROL[0]]
    assert not isinstance(out, str), out
    rc, tail = out
    assert rc == 0, f"the unchanged copy fails its pins (exit {rc})\n{tail}"
    assert " passed" in tail, tail


@pytest.mark.slow
@pytest.mark.parametrize("name", [p[0] for p in PLANTS])
def test_planted_mistake_fails_a_pin(outcomes, name):
    if name not in outcomes:
        pytest.skip("hipcc is not available to build the rocRAND cross-check")
    out = outcomes[name]
    assert not isinstance(out, str), f"{name}: {out}"
    rc, tail = out
    # pytest's exit status 1: tests ran and at least one failed (2-5: errors, no tests)
    assert rc == 1, f"{name}: the pins did not fail (exit {rc})\n{tail}"
    assert " failed" in tail, tail
