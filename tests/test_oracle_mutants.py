"""The oracle's pins must reject plausible mistakes.  Each case plants one
mistake in a copy of the oracle source (on the CPU), builds it, and checks that
the pin tests fail against it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "eifmm_oracle.c")

MUTANTS = {
    "lhat_uses_delta_not_delta_t": (
        "apply_delta_t(P->lv[k].a.d, P->dmax, P->lv[k].a.B, P->lv[k].a.G, v, w);",
        "apply_delta(P->lv[k].a.d, P->dmax, P->lv[k].a.B, P->lv[k].a.G, v, w);"),
    "two_eim_lhat_transposed": (
        "apply_delta(P->lv[k].b.d, P->dmax, P->lv[k].b.B, P->lv[k].b.G, v, w);",
        "apply_delta_t(P->lv[k].b.d, P->dmax, P->lv[k].b.B, P->lv[k].b.G, v, w);"),
    "two_eim_m2l_rows_from_first_eim": ("return P->two ? P->lv[k].b.X : P->lv[k].a.Y;",
                                        "return P->two ? P->lv[k].a.Y : P->lv[k].a.Y;"),
    "two_eim_l2p_points_from_first_eim": ("return P->two ? P->lv[k].b.Y : P->lv[k].a.X;",
                                          "return P->two ? P->lv[k].a.X : P->lv[k].a.X;"),
    "swapped_eim_keeps_roles": ("  if (swap) {\n    double *t = tx;", "  if (0) {\n    double *t = tx;"),
    "m2m_child_shift_sign": ("double xm[3] = {lv->X[3 * m] - sh[0]",
                             "double xm[3] = {lv->X[3 * m] + sh[0]"),
    "m2l_offset_sign": ("double yl[3] = {lv->Y[3 * ll] + dv[0]",
                        "double yl[3] = {lv->Y[3 * ll] - dv[0]"),
    "p2m_centre_sign": ("double yc[3] = {ps[3 * j] - c[0]", "double yc[3] = {ps[3 * j] + c[0]"),
    "gamma_recursion_sign": ("Gm[k * dmax + l] = s; /* unit", "Gm[k * dmax + l] = -s; /* unit"),
    "near_field_keeps_self": (
        "if (sing && zx == 0.0 && zy == 0.0 && zz == 0.0) continue;\n            s += ss[j]",
        "if (0) continue;\n            s += ss[j]"),
    "interaction_list_parent_rule": ("if (!inside || pc > 1) continue;",
                                     "if (!inside || pc > 2) continue;"),
    "two_eim_compression_columns_use_row_basis": ("const double *Vr = lvl->V ? lvl->V : lvl->U;",
                                                  "const double *Vr = lvl->U;"),
    "stage2_second_factor_transposed": ("t += Vo[(size_t)j * r + ll] * wj[ll];",
                                        "t += Vo[(size_t)ll * so + j] * wj[ll];"),
    "cosr_phase_uses_r_squared": ("return cos(K->p[0] * r) / r;",
                                  "return cos(K->p[0] * r2) / r;"),
    "mq_constant_outside_root": ("return sqrt(r2 + K->p[0]);", "return sqrt(r2) + K->p[0];"),
    "volume_kernels_trained_on_surfaces": ("static int kernel_is_volume(int kind) {\n  return !(",
                                           "static int kernel_is_volume(int kind) {\n  return 0 && !("),
}


def _run_mutant(name, base):
    """Build the oracle with mutant `name` planted and run the pin tests on it;
    returns (exit status, tail of the output)."""
    a, b = MUTANTS[name]
    src = open(SRC).read()
    d = base / name
    d.mkdir()
    mut = d / "mut.c"
    mut.write_text(src.replace(a, b, 1))
    so = d / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c99",
                    "-D_DEFAULT_SOURCE", "-o", str(so), str(mut), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(so), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_direct.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pass.py"),
                        os.path.join(ROOT, "tests", "test_oracle_eim.py"),
                        os.path.join(ROOT, "tests", "test_oracle_nonsym.py"),
                        os.path.join(ROOT, "tests", "test_oracle_compress2.py"),
                        "-k", "hand_values or finite_rank or gamma or interpolation or c1_accuracy "
                              "or swapped or two_eim or advdiff_two or stage2 or sides_random "
                              "or heldout"],
                       env=env, capture_output=True, text=True, cwd=ROOT)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def mutant_runs(tmp_path_factory):
    """All mutants at once, a few processes side by side (2 OpenMP threads each)."""
    from concurrent.futures import ThreadPoolExecutor
    base = tmp_path_factory.mktemp("mutants")
    names = sorted(MUTANTS)
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(workers) as ex:
        return dict(zip(names, ex.map(lambda n: _run_mutant(n, base), names)))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_runs):
    assert MUTANTS[name][0] in open(SRC).read()
    rc, out = mutant_runs[name]
    # 1: a pin test failed (or a crash); 0: all passed; 5: nothing was collected
    assert rc not in (0, 5), f"mutant {name} survived (status {rc}):\n{out}"
