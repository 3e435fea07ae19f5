"""CPU checks of the C ABI: the built library loads, exports every function include/dogm.h
declares, and its host-side logic (parameter validation, arena sizing, status strings) behaves
as documented.  No call here touches a GPU."""
import ctypes as ct
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dogm.h")


@pytest.fixture(scope="module")
def dl():
    from paper_1605_02406_amd import dogm
    if not os.path.exists(dogm.LIB_PATH):
        from paper_1605_02406_amd import build
        build.build()
    return dogm


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dogm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_abi(dl):
    assert declared_functions() == sorted(dl.ABI)


def test_library_exports_every_declared_symbol(dl):
    out = subprocess.run(["nm", "-D", "--defined-only", dl.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (dogm_[a-z_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported
    lib = dl.lib()
    for name in declared_functions():
        assert getattr(lib, name) is not None


def test_library_targets_gfx950_only(dl):
    """The library's embedded device code objects are all for gfx950."""
    data = open(dl.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-+(gfx[0-9a-z]+)", data))
    assert targets == {b"gfx950"}


def test_arena_bytes_and_validation(dl):
    p = dl.make_params(64, 64, 0.2, 32768, 8192)
    n = dl.arena_bytes(p)
    # at least the particle state (x..w, key) and the sorted copy
    assert n > 32768 * 4 * 13 + 4096 * 40
    p2 = dl.make_params(512, 512, 0.2, 2 ** 21, 2 ** 18)
    n2 = dl.arena_bytes(p2)
    assert n2 > 8 * n
    bad = [dict(nx=0), dict(cell_size=0.0), dict(cell_size=float("nan")), dict(p_s=1.5),
           dict(p_b=-0.1), dict(alpha_free=2.0), dict(n_pers=0), dict(n_born=-1),
           dict(n_pers=2 ** 27), dict(sigma_pos=-1.0), dict(nx=4096, ny=4096),
           dict(precision=2), dict(sort_passes=1), dict(sort_passes=4), dict(scan_parts=3),
           dict(resample=3)]
    for kw in bad:
        args = dict(nx=64, ny=64, cell_size=0.2, n_pers=32768, n_born=8192)
        args.update(kw)
        q = dl.make_params(**args)
        with pytest.raises(dl.DogmError) as e:
            dl.arena_bytes(q)
        assert e.value.code == dl.DOGM_EINVAL
    # launch plans: 64x64 keys need two passes of at most 11 bits; three are allowed
    for sp in (0, 2, 3):
        assert dl.arena_bytes(dl.make_params(64, 64, 0.2, 100, 10, sort_passes=sp)) > 0
    # the largest sizes the boundary accepts
    assert dl.arena_bytes(dl.make_params(4096, 4095, 0.2, 16, 0)) > 0
    assert dl.arena_bytes(dl.make_params(8, 8, 0.2, 2 ** 27 - 1, 0)) > 0
    q = dl.make_params(64, 64, 0.2, 10, 0)
    q.model = 2  # neither the Dempster-Shafer nor the particle PHD/MIB model
    with pytest.raises(dl.DogmError):
        dl.arena_bytes(q)
    q.model = dl.MODEL_PHD_MIB
    assert dl.arena_bytes(q) > 0


def test_null_handles_are_rejected(dl):
    lib = dl.lib()
    assert lib.dogm_predict(None) == dl.DOGM_EINVAL
    assert lib.dogm_step(None, None) == dl.DOGM_EINVAL
    assert lib.dogm_step_batch(None, None, 0, None) == dl.DOGM_OK  # empty batch
    assert lib.dogm_step_batch(None, None, -1, None) == dl.DOGM_EINVAL
    p = dl.make_params(8, 8, 0.2, 16, 4)
    h = ct.c_void_p()
    # a null or misaligned arena is rejected before anything touches a device
    assert lib.dogm_init_grid(ct.byref(p), None, 1 << 20, None, ct.byref(h)) == dl.DOGM_EINVAL
    assert lib.dogm_init_grid(ct.byref(p), ct.c_void_p(0x1001), 1 << 20, None,
                              ct.byref(h)) == dl.DOGM_EINVAL
    assert lib.dogm_init_grid(ct.byref(p), ct.c_void_p(0x100000), 16, None,
                              ct.byref(h)) == dl.DOGM_ESIZE
    assert dl.status_string(dl.DOGM_ESTATE) == "call out of order"
