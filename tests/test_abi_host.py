"""Host-side checks of the C ABI (no GPU needed): the built library exports every
function ``include/mbs.h`` declares, the Python binding's constants and struct
layouts match the header, and the argument validation and device-memory model
of ``mbs_plan_bytes`` behave as documented.  No call here launches a kernel.
"""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbs.h")


def _header():
    with open(HEADER) as fh:
        return fh.read()


def _declared_functions():
    text = re.sub(r"/\*.*?\*/", "", _header(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:mbs_status|const char\*)\s+(mbs_[a-z_]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def mbs_mod():
    from paper_2410_02395_amd import mbs
    if not os.path.exists(mbs.LIB_PATH):
        from paper_2410_02395_amd.build import build_library
        build_library(verbose=False)
    return mbs


@pytest.fixture(scope="module")
def lib(mbs_mod):
    return mbs_mod.load_library()


def test_library_exports_every_declared_function(mbs_mod, lib):
    declared = _declared_functions()
    assert len(declared) == 11
    assert sorted(mbs_mod.EXPORTS) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", mbs_mod.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_constants_match_header(mbs_mod):
    defs = dict(re.findall(r"#define\s+(MBS_[A-Z0-9_]+)\s+\(?(-?(?:0x)?[0-9a-fA-F]+)u?\)?", _header()))
    assert len(defs) >= 16
    for name, val in defs.items():
        assert getattr(mbs_mod, name) == int(val, 0), name


def test_struct_layouts_match_header(mbs_mod, tmp_path):
    """sizeof / offsetof of the ABI structs from a C compiler against the ctypes mirrors."""
    structs = {"mbs_plan_desc": mbs_mod.PlanDesc, "mbs_ramp": mbs_mod.Ramp, "mbs_result": mbs_mod.Result}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mbs.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def _desc(mbs, shape=(64, 64, 64), split=(1, 1, 1), periodic=(1, 1, 1), t=8, max_batch=1, alpha=0.75,
          check_every=0, flags=0, activation=0.0, zblock=0, reserved=0):
    d = mbs.PlanDesc()
    d.shape[:] = shape
    d.split[:] = split
    d.periodic[:] = periodic
    d.t = t
    d.max_batch = max_batch
    d.alpha = alpha
    d.flags = flags
    d.check_every = check_every
    d.activation = activation
    d.zblock = zblock
    d.reserved = reserved
    return d


def _bytes(mbs, lib, **kw):
    b = ctypes.c_size_t(0)
    st = lib.mbs_plan_bytes(ctypes.byref(_desc(mbs, **kw)), ctypes.byref(b))
    return st, b.value


def test_plan_bytes_memory_model(mbs_mod, lib):
    """Three complex64 arrays per voxel (iterate, work array, diagonal of I - V) plus
    4 t-deep edge buffers per corrected axis side pair, per slot; a fourth array when the
    slab schedule stores the work array slab by slab (arrays beyond the memory-side cache,
    power-of-two n_2: the 1024^3 plan); everything else is small and independent of the grid."""
    mbs = mbs_mod
    st, b1 = _bytes(mbs, lib, shape=(1024, 1024, 1024), split=(2, 2, 2), periodic=(0, 0, 0))
    assert st == mbs.MBS_OK
    vox, S, t, n = 1024 ** 3, 8, 8, 512
    slabs = 3 * S * 2 * t * n * n          # edge values per array kind, all three axes
    core = 32 * vox + 4 * 8 * slabs
    assert core <= b1 <= core + (64 << 20)
    # whole passes (no slabs), or slabs over an n_2 that is not a power of two: three arrays
    st, bw = _bytes(mbs, lib, shape=(1024, 1024, 1024), split=(2, 2, 2), periodic=(0, 0, 0), zblock=-1)
    assert st == mbs.MBS_OK and bw == b1 - 8 * vox
    st, bz = _bytes(mbs, lib, shape=(768, 768, 384), zblock=128)
    assert st == mbs.MBS_OK and 24 * 768 * 768 * 384 <= bz < 24 * 768 * 768 * 384 + (64 << 20)
    st, bp = _bytes(mbs, lib, shape=(512, 512, 512), zblock=128)
    assert st == mbs.MBS_OK and 32 * 512 ** 3 <= bp < 32 * 512 ** 3 + (64 << 20)
    st, b4 = _bytes(mbs, lib, shape=(1024, 1024, 1024), split=(2, 2, 2), periodic=(0, 0, 0), max_batch=4)
    assert st == mbs.MBS_OK and 4 * core <= b4 <= 4 * b1
    # a periodic single-domain grid has no edge buffers
    st, bp = _bytes(mbs, lib, shape=(256, 256, 256))
    assert st == mbs.MBS_OK and 24 * 256 ** 3 <= bp <= 24 * 256 ** 3 + (16 << 20)
    # the largest single-GPU grid of the plan's 2^31-voxel limit (four arrays per voxel with its
    # slab schedule) fits 288 GB of HBM with room
    st, big = _bytes(mbs, lib, shape=(2048, 1024, 1024), split=(4, 2, 2), periodic=(0, 0, 0))
    assert st == mbs.MBS_OK and big < 288e9 / 3


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(100, 64, 64)), "MBS_EUNSUPPORTED"),              # 100 = 2^2 5^2
    (dict(shape=(64, 64, 64), split=(3, 1, 1)), "MBS_EINVAL"),    # split does not divide
    (dict(shape=(2048, 64, 64)), "MBS_EUNSUPPORTED"),             # edge above 1024
    (dict(shape=(4, 64, 64)), "MBS_EUNSUPPORTED"),                # edge below 8
    (dict(shape=(64, 64, 64), split=(2, 1, 1), t=17), "MBS_EINVAL"),  # t above 16
    (dict(shape=(32, 64, 64), split=(2, 1, 1), t=9), "MBS_EINVAL"),   # t above n/2
    (dict(alpha=0.0), "MBS_EINVAL"),
    (dict(alpha=1.5), "MBS_EINVAL"),
    (dict(max_batch=0), "MBS_EINVAL"),
    (dict(check_every=-1), "MBS_EINVAL"),
    (dict(shape=(4096, 1024, 1024), split=(4, 1, 1)), "MBS_EUNSUPPORTED"),  # above 2^31 voxels
    (dict(activation=-1e-3), "MBS_EINVAL"),
    (dict(activation=float("nan")), "MBS_EINVAL"),
    # activation needs the fused z pass and at most 4096 subdomains
    (dict(shape=(64, 64, 64), split=(2, 2, 2), periodic=(0, 0, 0), flags=0x10, activation=1e-4),
     "MBS_EUNSUPPORTED"),
    (dict(shape=(512, 512, 16), split=(64, 64, 2), periodic=(0, 0, 0), t=4, activation=1e-4),
     "MBS_EUNSUPPORTED"),
    # z slabs of the strided passes: multiples of 16 (and of the tile width) dividing n_2
    (dict(zblock=-2), "MBS_EINVAL"),
    (dict(shape=(256, 256, 128), zblock=24), "MBS_EINVAL"),
    (dict(shape=(256, 256, 96), zblock=64), "MBS_EINVAL"),
    (dict(shape=(64, 64, 64), zblock=16), "MBS_EINVAL"),      # 64-point y pass: 32-column tiles
    (dict(shape=(256, 256, 128), zblock=32, flags=0x10), "MBS_EINVAL"),
    (dict(reserved=1), "MBS_EINVAL"),
])
def test_plan_bytes_rejects_what_plan_create_rejects(mbs_mod, lib, kw, status):
    st, _ = _bytes(mbs_mod, lib, **kw)
    assert st == getattr(mbs_mod, status)


def test_slab_heights_that_are_accepted(mbs_mod, lib):
    for zb in (-1, 0, 16, 32, 64, 128):
        st, _ = _bytes(mbs_mod, lib, shape=(256, 256, 128), zblock=zb)
        assert st == mbs_mod.MBS_OK, zb


def test_plan_bytes_with_activation(mbs_mod, lib):
    """Activation adds per-slot masks, lists and transfer partials: a few kB, not arrays."""
    kw = dict(shape=(1024, 1024, 1024), split=(2, 2, 2), periodic=(0, 0, 0), max_batch=2)
    st0, b0 = _bytes(mbs_mod, lib, **kw)
    st1, b1 = _bytes(mbs_mod, lib, activation=1e-4, **kw)
    assert st0 == st1 == mbs_mod.MBS_OK
    assert 0 < b1 - b0 < 64 << 10


def test_null_arguments_are_rejected_without_a_device(mbs_mod, lib):
    mbs = mbs_mod
    r = mbs.Result()
    assert lib.mbs_plan_bytes(None, None) == mbs.MBS_EINVAL
    assert lib.mbs_plan_bytes(ctypes.byref(_desc(mbs)), None) == mbs.MBS_EINVAL
    assert lib.mbs_plan_create(ctypes.byref(_desc(mbs)), None, None) == mbs.MBS_EINVAL
    assert lib.mbs_plan_destroy(None) == mbs.MBS_EINVAL
    assert lib.mbs_set_medium(None, 0, None, 1.0, None) == mbs.MBS_EINVAL
    assert lib.mbs_solve(None, 0, None, 0.0, 1, None, ctypes.byref(r)) == mbs.MBS_EINVAL
    assert lib.mbs_solve_async(None, 0, None, 0.0, 1, None) == mbs.MBS_EINVAL
    assert lib.mbs_poll(None, 0, ctypes.byref(r)) == mbs.MBS_EINVAL
    rel = ctypes.c_double()
    assert lib.mbs_residual(None, 0, None, ctypes.byref(rel)) == mbs.MBS_EINVAL
    n = ctypes.c_int32()
    assert lib.mbs_residual_history(None, 0, None, 0, ctypes.byref(n)) == mbs.MBS_EINVAL
    assert lib.mbs_timing_read(None, None, None, 8, 0) == mbs.MBS_EINVAL


def test_every_status_has_a_message(mbs_mod, lib):
    msgs = set()
    for code in range(0, -11, -1):
        m = lib.mbs_strerror(code).decode()
        assert m and m != "unknown status"
        msgs.add(m)
    assert len(msgs) == 11
    assert lib.mbs_strerror(-99).decode()
