"""The oracle's pins have teeth: plant plausible mistakes in copies of the
oracle source (on the CPU), rebuild, and require at least one pin to fail for
every planted mistake.  The real oracle is never modified."""

import pytest

import oracle
import oracle_pins as P

# (name, original text, planted text)
MUTANTS = [
    ("drop_half_in_log", "return 0.5 * log(lam) / fabs(T);", "return log(lam) / fabs(T);"),
    ("signed_T", "return 0.5 * log(lam) / fabs(T);", "return 0.5 * log(lam) / T;"),
    ("M_diagonal_only", "M[r][c] += dx[r] * dx[c];", "M[r][c] += (r == c) ? dx[r] * dx[c] : 0.0;"),
    ("transposed_rhs", "R[r][c] += dx[r] * df[c];", "R[r][c] += dx[c] * df[r];"),
    ("smaller_eigenvalue_2d", "st->lam = m + h;", "st->lam = m - h;"),
    ("jacobi_rotation_sign", "a[r][p] = a[p][r] = c * arp - s * arq;", "a[r][p] = a[p][r] = c * arp + s * arq;"),
    ("elimination_factor", "for (int k = c; k < D; ++k) A[r][k] -= f * A[c][k];",
     "for (int k = c; k < D; ++k) A[r][k] -= A[c][k];"),
    ("axis_least_aligned", "if (arg < 0 || cosang > best)", "if (arg < 0 || cosang < best)"),
    ("ring1_keeps_self", "if (v == (int32_t)i || v == prev) continue;", "if (v == prev) continue;"),
    ("adjoint_drop_self_term", "grad[i * D + r] -= s;", "(void)0;"),
    ("adjoint_transposed_G", "R[r][c] = coef * Jv[c] * st.v[r];", "R[r][c] = coef * Jv[r] * st.v[c];"),
    ("adjoint_no_inv_lambda", "double coef = g[i] / (fabs(T) * st.lam);", "double coef = g[i] / fabs(T);"),
    ("adjoint_wrong_eigvec_2d", "if (d >= 0.0) { v0 = d + h; v1 = b; }", "if (d >= 0.0) { v0 = b; v1 = d + h; }"),
]


@pytest.fixture(scope="module")
def workloads_small():
    from workloads import configs
    return configs.small_2d(), configs.abc3d(8, 10.0, "f64")


def _pins(lib, w2, w3):
    for check in P.ALL_BASIC:
        yield check.__name__, lambda check=check: check(lib=lib)
    yield "invariances", lambda: P.check_invariances(w2, w3, lib=lib)
    yield "relabel", lambda: P.check_relabel(w2, lib=lib)
    yield "adjoint_identities", lambda: P.check_adjoint_identities(lib=lib)
    yield "adjoint_fd", lambda: P.check_adjoint_fd(lib=lib, max_points=40)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new, tmp_path, workloads_small):
    src = open(oracle.source_path()).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/present"
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src.replace(old, new))
    so = oracle.compile_source(str(path), str(tmp_path / f"libmut_{name}.so"))
    lib = oracle.load_library(so)
    w2, w3 = workloads_small
    failed = []
    for pin, run in _pins(lib, w2, w3):
        try:
            run()
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(pin)
            break
    assert failed, f"planted mistake {name} passed every pin"
