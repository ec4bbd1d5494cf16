"""CPU-side checks of the C interface: the library loads and exports every
function the header declares; host-side helpers behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qmg.h")
LIB = os.path.join(ROOT, "paper_2004_08146_amd", "libqmg.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qmg_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("qmg_set_gauge", "qmg_apply_Q", "qmg_apply_Q_shifted", "qmg_sap_smooth",
                     "qmg_restrict", "qmg_prolong", "qmg_apply_coarse", "qmg_solve_shifted"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqmg.so not built")
def test_binding_covers_every_symbol():
    from paper_2004_08146_amd import qmg
    assert sorted(qmg.EXPORTED) == _declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqmg.so not built")
def test_default_params_follow_parameter_table():
    from paper_2004_08146_amd import qmg
    p = qmg.default_params()
    assert p.coarse_tol == 0.5          # coarse grid tolerance 5e-1 (parameter table)
    assert p.tol == 1e-10
    assert p.nu_post == 3 and p.n_mr == 3
    q = qmg.default_params(mg_prec="bf16", restart=8)
    assert q.mg_prec == qmg.BF16 and q.restart == 8
