"""Host-only checks of the C ABI: the library loads, exports every function
include/spme.h declares, and rejects bad arguments before touching a device.
The product package never imports the oracle."""
import ctypes
import os
import re

import pytest

from paper_2009_12617_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2009_12617_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2009_12617_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2009_12617_amd import _lib
    names = _lib.declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert lib.pme_version() >= 100


def test_workspace_bytes(lib):
    w = lib.pme_workspace_bytes(64, 64, 64, 4, 65535, 1)
    assert w > 0 and w % 256 == 0
    # the workspace holds at least the half spectrum and the potential
    assert w > 64 * 64 * 33 * 8 + 64 ** 3 * 4
    w64 = lib.pme_workspace_bytes(64, 64, 64, 4, 65535, 0)
    assert w64 > 64 * 64 * 33 * 16 + 64 ** 3 * 8
    assert lib.pme_workspace_bytes(50, 50, 50, 4, 100, 1) == 0      # radix 5
    assert lib.pme_workspace_bytes(64, 64, 32, 4, 100, 1) == 0      # shape without kernels
    assert lib.pme_workspace_bytes(64, 32, 64, 4, 100, 1) == 0
    # non-cubic shapes with kernels: the spectrum [K1/2+1][K3][K2] and the
    # potential rows [K3][K2] scale with the shape
    wn = lib.pme_workspace_bytes(64, 64, 128, 4, 65535, 1)
    assert wn > 64 * 128 * 33 * 8 + 64 * 64 * 128 * 4
    assert lib.pme_workspace_bytes(32, 32, 64, 6, 1000, 0) > 0
    assert lib.pme_workspace_bytes(48, 32, 64, 4, 1000, 2) > 0
    assert lib.pme_workspace_bytes(64, 64, 64, 5, 100, 1) == 0      # odd order
    assert lib.pme_workspace_bytes(64, 64, 64, 4, -1, 1) == 0
    assert lib.pme_workspace_bytes(64, 64, 64, 4, 100, 7) == 0
    # the two reduced-precision spectra store 4 bytes per complex value, so
    # their workspaces agree; where the split convolution is available
    # (every shape here) they also hold the full-precision intermediate
    # between its passes: half spectrum points x (4 + 8) bytes in place of 8
    for g in ((64, 64, 64), (64, 64, 128)):
        wh = lib.pme_workspace_bytes(*g, 4, 65535, 2)
        assert wh > 0 and lib.pme_workspace_bytes(*g, 4, 65535, 3) == wh
        half = g[1] * g[2] * (g[0] // 2 + 1)
        assert abs(wh - (lib.pme_workspace_bytes(*g, 4, 65535, 1) + 4 * half)) <= 512


def create(lib, K=32, order=4, beta=0.35, max_atoms=100, prec=1, frac=0, coul=0.0,
           ws=None, nbytes=None):
    h = ctypes.c_void_p()
    if nbytes is None:
        nbytes = 1 << 30
    rc = lib.pme_create(ctypes.byref(h), K, K, K, order, beta, max_atoms, prec, frac, coul,
                        ws, nbytes, None)
    return rc, h


def test_create_rejects_bad_arguments_without_a_device(lib):
    fake = 0x7f0000000000  # never dereferenced: validation happens first
    assert create(lib, beta=0.0, ws=fake)[0] == 1
    assert create(lib, beta=float("nan"), ws=fake)[0] == 1
    assert create(lib, max_atoms=-5, ws=fake)[0] == 1
    assert create(lib, prec=4, ws=fake)[0] == 1  # 0..3 are the precisions
    assert create(lib, frac=50, ws=fake)[0] == 1
    assert create(lib, coul=float("inf"), ws=fake)[0] == 1
    assert create(lib, K=50, ws=fake)[0] == 2
    assert create(lib, order=5, ws=fake)[0] == 2
    assert create(lib, order=8, ws=fake)[0] == 2
    assert create(lib, ws=None)[0] == 3
    assert create(lib, ws=fake + 8)[0] == 3           # misaligned
    assert create(lib, ws=fake, nbytes=1024)[0] == 3  # too small
    rc, h = create(lib, beta=0.0, ws=fake)
    assert h.value is None
    assert lib.pme_create(None, 32, 32, 32, 4, 0.3, 1, 1, 0, 0.0, fake, 1 << 30, None) == 1


def test_null_plan_calls_are_rejected(lib):
    box = (ctypes.c_double * 9)(20, 0, 0, 0, 20, 0, 0, 0, 20)
    assert lib.pme_spread(None, None, None, 0, box) == 1
    assert lib.pme_solve(None, None) == 1
    assert lib.pme_gather(None, None, 0) == 1
    assert lib.pme_step(None, None, None, 0, box, None, 0, None) == 1
    assert lib.pme_destroy(None) == 1
    assert lib.pme_check(None, None) == 1
    assert lib.pme_debug_grid_bytes(None, 0) == 0
    for code in range(9):
        assert lib.pme_strerror(code) != b"unknown status"
    assert lib.pme_strerror(99) == b"unknown status"


def test_product_package_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2009_12617_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "spme_oracle" not in text, f
                assert "liboracle" not in text, f


def test_noalloc_step_answers_without_a_device(lib):
    # the size limit and argument checks answer before any device work
    fake = 0x7f0000000000
    box = (ctypes.c_double * 9)(128, 0, 0, 0, 128, 0, 0, 0, 128)
    need = lib.pme_workspace_bytes(128, 128, 128, 4, 209715, 1)
    assert need > _lib.PME_SCRATCH_BYTES
    assert lib.pme_step_noalloc(128, 128, 128, 4, 0.32, 1, 0, 0.0, fake, fake, 209715, box,
                                fake, 0, fake, None) == 3          # PME_EWORKSPACE
    assert lib.pme_workspace_bytes(64, 64, 64, 4, 65536, 1) <= _lib.PME_SCRATCH_BYTES
    assert lib.pme_step_noalloc(64, 64, 64, 4, 0.0, 1, 0, 0.0, fake, fake, 100, box,
                                fake, 0, fake, None) == 1          # beta
    assert lib.pme_step_noalloc(50, 50, 50, 4, 0.3, 1, 0, 0.0, fake, fake, 100, box,
                                fake, 0, fake, None) == 2          # radix 5
    assert lib.pme_step_noalloc(64, 64, 64, 4, 0.3, 1, 0, 0.0, fake, fake, 100, None,
                                fake, 0, fake, None) == 1          # no box
    assert lib.pme_step_noalloc(64, 64, 64, 4, 0.3, 1, 0, 0.0, fake, fake, 100, box,
                                None, 0, fake, None) == 1          # no forces
