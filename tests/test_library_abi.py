"""CPU checks of the C ABI library: it builds, loads and exports every symbol
declared in include/kerrhip.h; host-only helpers return sane values."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("kerrhip.h", "kerrhip_mlp.h")]
LIB = os.path.join(ROOT, "paper_1706_07062_amd", "libkerrhip.so")


def declared_symbols():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kh_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1706_07062_amd import build as B

        B.build()
    return C.CDLL(LIB)


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("kh_create", "kh_destroy", "kh_init_rays", "kh_integrate", "kh_read_state", "kh_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_1706_07062_amd as K

    assert sorted(K.EXPORTS + K.MLP_EXPORTS) == declared_symbols()


def test_default_params_and_struct_layout():
    import paper_1706_07062_amd as K

    p = K.kh_default_params()
    assert p.method == K.DOPRI5 and p.precision == K.P64
    assert p.rtol == 1e-8 and p.atol == 1e-8 and p.h_coeff == 0.01 and p.hmax_coeff == 0.1
    assert p.r_h_factor == 1.01 and p.r_escape == 1000.0 and p.max_steps == 1_000_000
    # struct sizes agree with the C layout (8-byte aligned doubles)
    assert C.sizeof(K.kh_camera) == 64
    assert C.sizeof(K.kh_params) == 112
    assert C.sizeof(K.kh_state) == 8 * 20
    assert C.sizeof(K.kh_flop_counts) == 8 * 9
    assert C.sizeof(K.kh_fixed_params) == 16 + 8 * 4


def test_flop_counts():
    import paper_1706_07062_amd as K

    f = K.kh_flops(K.DOPRI5, K.RHS_FACTORED)
    p = K.kh_flops(K.DOPRI5, K.RHS_PAPER)
    rhs_f = f["add"] + f["mul"] + f["div"] + f["sqrt"]
    rhs_p = p["add"] + p["mul"] + p["div"] + p["sqrt"]
    # both forms take one square root (radius root), one reciprocal square root
    # (r and 1/r) and one reciprocal (1/S and 1/D from 1/(S D))
    assert f["sqrt"] == 2 and p["sqrt"] == 2
    assert f["div"] == 1 and p["div"] == 1
    assert 80 < rhs_f < rhs_p < 400
    # a DOPRI5 attempt adds the stage combinations and the error norm; the
    # norm stays squared (the controller works with err^2), so no square root
    assert f["step_add"] > 100 and f["step_mul"] > 100 and f["step_sqrt"] == 0
    r = K.kh_flops(K.RK4, K.RHS_FACTORED)
    assert r["step_add"] > 20
    assert f["trig"] == 0 and r["trig"] == 0
    # Boyer-Lindquist form: one sin and one cos, one reciprocal (1/rho^2,
    # 1/Delta, 1/sin^2 from their product), no root; the same RK4 step
    b = K.kh_flops(K.RK4, K.RHS_BL)
    assert b["trig"] == 2 and b["sqrt"] == 0 and b["div"] == 1
    assert 80 < b["add"] + b["mul"] < 400
    assert (b["step_add"], b["step_mul"]) == (r["step_add"], r["step_mul"])
    with pytest.raises(K.KerrHipError):
        K.kh_flops(K.DOPRI5, K.RHS_BL)
