"""The pins are strong enough to catch plausible mistakes in the oracle.

Each case plants one mistake (a wrong sign, a dropped term, a wrong index, a
transposed operand) in a private copy of oracle.c, compiles it on the CPU,
swaps it in for the real oracle, and checks that the named pin now fails.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_1d as t1
import test_oracle_2d as t2
import test_oracle_adjoint as ta

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = [
    ("1d sign of right neighbour", "return uc + r * ((ul - 2.0 * uc) + ur);",
     "return uc + r * ((ul - 2.0 * uc) - ur);",
     lambda: t1.test_periodic_matches_spectral_closed_form(64, 0.1, 40)),
    ("1d dirichlet wraps", "double ur = (i == n - 1) ? 0.0 : a[i + 1];",
     "double ur = a[(i + 1) % n];",
     lambda: t1.test_dirichlet_matches_dst_closed_form(31, 0.25, 20)),
    ("2d centre weight", "b[i * nx + j] = c + r * (((n_ + s_) + (w_ + e_)) - 4.0 * c);",
     "b[i * nx + j] = c + r * (((n_ + s_) + (w_ + e_)) - 3.0 * c);",
     lambda: t2.test_dirichlet2d_matches_dst_closed_form(7, 9, 0.25, 10)),
    ("2d dropped south neighbour",
     "double s_ = (i < ny - 1) ? a[(i + 1) * nx + j] : 0.0;", "double s_ = 0.0;",
     lambda: t2.test_dirichlet2d_separable_mode()),
    ("face conductivity not averaged", "return 0.5 * (kc + kappa[*nb]);", "return kc;",
     lambda: t2.test_varcoef_operator_symmetric_and_linear_in_kappa()),
    ("edge face uses neighbour conductivity rule",
     "if (ni < 0 || ni >= ny || nj < 0 || nj >= nx) { *nb = -1; return kc; }",
     "if (ni < 0 || ni >= ny || nj < 0 || nj >= nx) { *nb = -1; return 0.5 * kc; }",
     lambda: t2.test_varcoef_hand_computed_1x2()),
    ("transpose scatters the wrong cell", "lam_out[nb] = lam_out[nb] + (dt * kf) * lam_in[m];",
     "lam_out[nb] = lam_out[nb] + (dt * kf) * lam_in[nb];",
     lambda: ta.test_inner_product_identity(16, 16)),
    ("edge-face gradient sign", "acc = acc + u_t[c] * lam_next[c];",
     "acc = acc - u_t[c] * lam_next[c];", lambda: ta.test_fd_in_kappa_every_cell()),
    ("interior-face gradient missing half",
     "acc = acc + 0.5 * ((u_t[nb] - u_t[c]) * (lam_next[nb] - lam_next[c]));",
     "acc = acc + ((u_t[nb] - u_t[c]) * (lam_next[nb] - lam_next[c]));",
     lambda: ta.test_closed_form_single_mode()),
    ("adjoint seed without target", "for (size_t c = 0; c < cells; ++c) lam[c] = cur[c] - y[c];",
     "for (size_t c = 0; c < cells; ++c) lam[c] = cur[c];",
     lambda: ta.test_fd_in_u0_is_exact_for_quadratic_loss()),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(tmp_path, monkeypatch, name, old, new, pin):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique/absent: {old}"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                           str(lib), str(mpath), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle._bind(str(lib)))
    with pytest.raises(AssertionError):
        pin()
