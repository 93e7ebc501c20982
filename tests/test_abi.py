"""The C ABI library loads and exports every symbol include/qla.h declares (no GPU
needed); argument checks that return before any device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qla.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qla_[a-z_]+)\s*\(", text)))


def _lib():
    from paper_2604_21128_amd import qla
    if not os.path.exists(qla.LIB_PATH):
        pytest.fail("libqla.so is not built (run `python -m paper_2604_21128_amd.build`)")
    return qla, qla.load()


def test_header_declares_the_documented_calls():
    names = _declared()
    for must in ("qla_create", "qla_set_index", "qla_init_packet", "qla_advance",
                 "qla_get_fields", "qla_energy", "qla_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    qla, lib = _lib()
    declared = _declared()
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(qla.EXPORTED) == declared


def test_status_strings():
    qla, _ = _lib()
    assert qla.qla_strerror(qla.QLA_OK) == "success"
    assert qla.qla_strerror(qla.QLA_EINVAL) == "invalid argument"
    assert qla.qla_strerror(qla.QLA_ESTATE) == "call out of order"


@pytest.mark.parametrize("nx,ny,delta,prec,pot", [
    (4, 64, 0.25, 0, 0),       # lattice too small for the 4-cell neighbourhood
    (64, 7, 0.25, 0, 0),
    (64, 64, 0.0, 0, 0),       # delta must be > 0
    (64, 64, float("nan"), 0, 0),
    (64, 64, 0.25, 7, 0),      # bad precision
    (64, 64, 0.25, 0, 9),      # bad potential mode
    (64, 64, 0.25, 0, 4),
    (1 << 28, 8, 0.25, 0, 0),    # a row of 2 GiB or more
])
def test_create_rejects_bad_arguments_before_touching_the_device(nx, ny, delta, prec, pot):
    qla, lib = _lib()
    out = ctypes.c_void_p(1234)
    st = lib.qla_create(nx, ny, delta, prec, pot, None, ctypes.byref(out))
    assert st == qla.QLA_EINVAL
    assert out.value is None
    assert qla.qla_last_error()


def test_null_context_is_rejected():
    qla, lib = _lib()
    assert lib.qla_advance(None, 1) == qla.QLA_EINVAL
    assert lib.qla_energy(None, None) == qla.QLA_EINVAL
    assert lib.qla_destroy(None) == qla.QLA_OK


@pytest.mark.parametrize("args", [
    (32, 32, 4, 3, 16, 17, 2, 32, 2),     # 2 * modes > height
    (32, 20, 4, 3, 16, 12, 2, 32, 2),     # 2 * modes > width
    (32, 32, 0, 3, 16, 4, 2, 32, 2),      # no input channels
    (32, 32, 4, 3, 16, 4, 0, 32, 2),      # no layers
    (32, 32, 4, 3, 16, 4, 2, 32, 0),      # no batch
    (32, 32, 4, 3, 65, 4, 2, 32, 2),      # width beyond 64
    (8192, 8192, 4, 3, 64, 12, 4, 128, 4),  # activations beyond 2^31 elements
])
def test_surrogate_create_rejects_bad_sizes_before_touching_the_device(args):
    qla, lib = _lib()
    out = ctypes.c_void_p(1234)
    st = lib.qla_fno_create(*args, 0, None, ctypes.byref(out))
    assert st == qla.QLA_EINVAL
    assert out.value is None


def test_surrogate_null_handle_is_rejected():
    qla, lib = _lib()
    assert lib.qla_fno_forward(None, None, 1, None) == qla.QLA_EINVAL
    assert lib.qla_fno_adam_step(None, 1e-3, 0.9, 0.999, 1e-8) == qla.QLA_EINVAL
    assert lib.qla_fno_param_count(None, None) == qla.QLA_EINVAL
    assert lib.qla_fno_band_fraction(None, None, 1, 1, 3, None) == qla.QLA_EINVAL
    assert lib.qla_fno_destroy(None) == qla.QLA_OK


def test_bz_triple_rejects_the_printed_potentials_and_bad_triples():
    qla, lib = _lib()
    out = ctypes.c_void_p(1234)
    assert lib.qla_create_triple(64, 64, 0.25, 0, qla.QLA_V_PAPER, qla.QLA_TRIPLE_BZ, None,
                                 ctypes.byref(out)) == qla.QLA_EINVAL
    assert lib.qla_create_triple(64, 64, 0.25, 0, 0, 7, None, ctypes.byref(out)) == qla.QLA_EINVAL
    assert lib.qla_create_triple(64, 64, 0.25, 0, qla.QLA_V_BSTREAM, qla.QLA_TRIPLE_BZ, None,
                                 ctypes.byref(out)) == qla.QLA_EINVAL
    assert lib.qla_divergence(None, None, None, None) == qla.QLA_EINVAL


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: without the built library the binding raises instead of
    computing anything (checked in a fresh interpreter, the library not yet loaded)."""
    import subprocess
    import sys
    missing = str(tmp_path / "libqla.so")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2604_21128_amd import qla\n"
            "qla.LIB_PATH = %r\n"
            "try:\n"
            "    qla.load(%r)\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n"
            "else:\n"
            "    print('loaded')\n") % (ROOT, missing, missing)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("raised") and "not built" in out.stdout
