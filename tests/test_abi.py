"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import os
import re

import pytest

from paper_2301_08275_amd import gpe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gpe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gpe_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gpe_create", "gpe_evolve", "gpe_ground_state", "gpe_observables",
                 "gpe_destroy", "gpe_last_error", "gpe_spectra_bins"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gpe.LIB_PATH):
        pytest.fail("libgpe.so is not built; run __graft_entry__.build() first")
    lib = gpe.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in gpe.SIGNATURES, name


def test_binding_covers_exactly_the_header():
    assert sorted(gpe.SIGNATURES) == declared_functions()


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        gpe._lib_saved = gpe._lib
        try:
            gpe._lib = None
            gpe.load_library(str(tmp_path / "nope.so"))
        finally:
            gpe._lib = gpe._lib_saved


def test_header_is_plain_c(tmp_path):
    """include/gpe.h compiles as C99 (the boundary is a C ABI, not C++)."""
    import subprocess

    src = os.path.join(ROOT, "tests", "c", "abi_demo.c")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), src], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _unbound_context(shape=(8, 8)):
    """A Context object with no library context behind it: only the host-side
    argument checks can run on it."""
    ctx = gpe.Context.__new__(gpe.Context)
    ctx.shape, ctx.dim, ctx._ctx, ctx._own_stream, ctx._vfn = tuple(shape), len(shape), None, True, None
    return ctx


@pytest.mark.parametrize("make", [
    lambda torch: torch.zeros((8, 8), dtype=torch.complex128),      # host tensor
    lambda torch: torch.zeros((8, 8), dtype=torch.float64),         # real dtype
    lambda torch: torch.zeros((8, 8, 2), dtype=torch.float32),      # real dtype, other shape
    lambda torch: torch.zeros((8, 8), dtype=torch.complex64),       # host tensor, FP32
])
def test_device_state_calls_reject_bad_tensors_before_any_library_call(make):
    """set_state_device / get_state_device hand a raw device pointer to the
    library: a host tensor or a real-valued one must raise before that."""
    torch = pytest.importorskip("torch")
    ctx = _unbound_context()
    t = make(torch)
    with pytest.raises(ValueError):
        ctx.set_state_device(t)
    with pytest.raises(ValueError):
        ctx.get_state_device(t)
