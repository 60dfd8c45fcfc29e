"""The C ABI library loads and exports every function include/demons.h declares.

No GPU is needed: only host-side entry points are called (version, strings,
timing names, NULL-handle argument checks).
"""
import ctypes
import os
import re
import subprocess
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "demons.h")
LIB = os.path.join(ROOT, "paper_0909_0928_amd", "libdemons.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdemons.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dir_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dir_create", "dir_register", "dir_warp", "dir_destroy", "dir_strerror", "dir_force",
                     "dir_smooth", "dir_gradient", "dir_restrict", "dir_prolong", "dir_compose"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (dir_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported


def test_host_only_entry_points():
    from paper_0909_0928_amd import binding as B
    L = B.lib()
    assert L.dir_abi_version() == 1
    assert B.dir_strerror(0) == "success"
    assert B.dir_strerror(-1) == "invalid argument"
    assert B.dir_strerror(12345) == "unknown status code"
    names = B.dir_timing_names()
    assert "force" in names and "smooth_x" in names and len(names) == L.dir_timing_count()
    assert L.dir_timing_name(-1) is None and L.dir_timing_name(len(names)) is None
    assert L.dir_timing_read(None, 0, None, None) == B.DIR_EINVAL
    assert L.dir_timing_read_level(None, 0, 0, None, None) == B.DIR_EINVAL
    # NULL handle: rejected before any device call
    assert L.dir_warp(None, None, None, 4, 4, 4, None) == B.DIR_EINVAL
    assert L.dir_register(None, None, None, 4, 4, 4, None, None, None, None) == B.DIR_EINVAL
    assert L.dir_destroy(None) == B.DIR_OK
    assert L.dir_create(None, 0, None) == B.DIR_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    from paper_0909_0928_amd import binding as B
    src = tmp_path / "sizes.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "demons.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dir_params), sizeof(dir_stats),'
                   'offsetof(dir_params, iters), offsetof(dir_params, eps), offsetof(dir_stats, history),'
                   'offsetof(dir_stats, history_len), offsetof(dir_params, units), offsetof(dir_params, image_sigma));'
                   ' return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(s) for s in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert sizes == [ctypes.sizeof(B.dir_params), ctypes.sizeof(B.dir_stats), B.dir_params.iters.offset,
                     B.dir_params.eps.offset, B.dir_stats.history.offset, B.dir_stats.history_len.offset,
                     B.dir_params.units.offset, B.dir_params.image_sigma.offset]
    assert sizes[0] == 96   # no implicit padding (graph keys compare parameters bytewise)


def test_workspace_bytes_accounting():
    """dir_workspace_bytes follows the buffers a registration allocates."""
    from paper_0909_0928_amd import binding as B
    shape = (32, 64, 64)
    n = 32 * 64 * 64
    one = lambda v, st: B.dir_workspace_bytes(shape, B.make_params(v, [50], sigma=1.0, storage=st))
    # 16-bit storage: two fields of 3N values at 2 B instead of 4, plus 2 B copies of S and M
    assert one("passive", "f32") - one("passive", "f16") == 2 * 3 * n * 2 - 2 * 2 * n
    assert one("passive", "bf16") == one("passive", "f16")
    # active keeps D (storage format); IC keeps D and P (FP32)
    assert one("active", "f32") - one("passive", "f32") == 4 * n
    assert one("inverse_consistent", "f32") - one("passive", "f32") == 8 * n
    assert one("inverse_consistent", "f16") - one("passive", "f16") == 2 * n + 4 * n
    # pyramid levels: S and M at every coarser level (ceil halving)
    two = B.dir_workspace_bytes(shape, B.make_params("passive", [25, 25], sigma=1.0))
    assert two - one("passive", "f32") == 2 * 4 * (16 * 32 * 32)
    # image pre-smoothing keeps a smoothed copy of every level of S and M
    pre = B.dir_workspace_bytes(shape, B.make_params("passive", [25, 25], sigma=1.0, image_sigma=1.0))
    assert pre - two == 2 * 4 * (n + 16 * 32 * 32)
    pre16 = B.dir_workspace_bytes(shape, B.make_params("passive", [50], sigma=1.0, image_sigma=1.0, storage="f16"))
    assert pre16 - one("passive", "f16") == 2 * 2 * n
    # physical units need no extra buffers
    assert B.dir_workspace_bytes(shape, B.make_params("passive", [50], sigma=1.0, units="mm")) == one("passive", "f32")
    bad = B.make_params("passive", [5], sigma=1.0)
    bad.sigma = -1.0
    with pytest.raises(B.DemonsError):
        B.dir_workspace_bytes(shape, bad)
    for field, value in (("image_sigma", -0.5), ("image_sigma", float("nan")), ("units", 2), ("units", -1)):
        bad = B.make_params("passive", [5], sigma=1.0)
        setattr(bad, field, value)
        with pytest.raises(B.DemonsError):
            B.dir_workspace_bytes(shape, bad)
    # voxel units: the pre-smoothing radius ceil(3 image_sigma) must stay within 16
    with pytest.raises(B.DemonsError):
        B.dir_workspace_bytes(shape, B.make_params("passive", [5], sigma=1.0, image_sigma=5.5))


def test_size_limit_and_empty_volumes():
    """Buffers are addressed with 32-bit byte ranges: a 3-component FP32 field
    must stay below 4 GiB, so nx*ny*nz <= 357,913,941; empty volumes are
    rejected."""
    from paper_0909_0928_amd import binding as B
    p = B.make_params("passive", [1], sigma=1.0)
    assert B.dir_workspace_bytes((1, 1, 357913941), p) > 12 * 357913941
    for shape in ((1, 1, 357913942), (1024, 1024, 342), (0, 4, 4), (4, 0, 4), (4, 4, 0), (4, -1, 4)):
        with pytest.raises(B.DemonsError):
            B.dir_workspace_bytes(shape, p)


def test_batch_and_pool_argument_checks():
    """Batch and pool entry points reject bad arguments before any device call."""
    from paper_0909_0928_amd import binding as B
    L = B.lib()
    assert B.DIR_MAX_BATCH == 8
    # NULL handle / pool
    assert L.dir_register_batch(None, 1, None, None, None, None, None, None, None) == B.DIR_EINVAL
    assert L.dir_register_batch_async(None, 1, None, None, None, None, None, None) == B.DIR_EINVAL
    assert L.dir_pool_set_max_batch(None, 2) == B.DIR_EINVAL
    assert L.dir_wait(None, None) == B.DIR_EINVAL
    # the binding checks list lengths and counts before touching the library
    p = B.make_params("passive", [2], sigma=1.0)
    h = B.Handle(None, 0)
    with pytest.raises(ValueError):
        B.dir_register_batch(h, [], [], [])
    with pytest.raises(ValueError):
        B.dir_register_batch(h, [None] * 9, [None] * 9, [p] * 9)
    with pytest.raises(ValueError):
        B.dir_register_batch(h, [None, None], [None], [p, p])
    with pytest.raises(ValueError):  # not GPU tensors
        B.dir_register_batch(h, [None], [None], [p])


def test_autotune_argument_checks():
    from paper_0909_0928_amd import binding as B
    L = B.lib()
    p = B.make_params("passive", [2], sigma=1.0)
    assert L.dir_autotune(None, 8, 8, 8, ctypes.byref(p), 1, None) == B.DIR_EINVAL
    B.dir_autotune_clear()  # host only


def test_noalloc_scratch_limit_is_checked_on_the_host():
    """dir_step_noalloc checks the scratch size it needs before it touches the
    handle or a device: with a NULL handle a volume beyond the array is refused
    with the size message, one within it only for the NULL handle."""
    from paper_0909_0928_amd import binding as B
    L = B.lib()
    text = open(HEADER).read()
    assert re.search(r"#define DIR_NOALLOC_SCRATCH_BYTES \(128u \* 1024u \* 1024u\)", text)
    assert B.DIR_NOALLOC_SCRATCH_BYTES == 128 * 1024 * 1024
    # addresses that are never dereferenced (every call returns before any
    # device work) and far enough apart that the field and output cannot overlap
    p, q = ctypes.c_void_p(1 << 44), ctypes.c_void_p(1 << 45)
    sums = (ctypes.c_double * 3)()

    def call(variant, nx, ny, nz):
        """Status and error message of one call, in a fresh thread (the
        message is per thread)."""
        res = []

        def run():
            rc = L.dir_step_noalloc(None, variant, 1.0, p, p, p, nx, ny, nz, 1.5, 5, q, sums)
            res.append((rc, B._last_error()))
        t = threading.Thread(target=run)
        t.start()
        t.join()
        return res[0]

    def need(variant, n, blocks):
        a = lambda b: (b + 255) // 256 * 256
        pre = variant in (B.DIR_ACTIVE, B.DIR_DOUBLE, B.DIR_INVERSE_CONSISTENT)
        return (a(8) + a(32) + a(24 * blocks) + a(12 * n) + (a(4 * n) if pre else 0)
                + (a(4 * n) if variant == B.DIR_INVERSE_CONSISTENT else 0))

    # 256x256x100: 6400 force workgroups; fits every variant
    for variant in range(5):
        assert need(variant, 256 * 256 * 100, 6400) <= B.DIR_NOALLOC_SCRATCH_BYTES
        assert call(variant, 256, 256, 100) == (B.DIR_EINVAL, "")   # refused for the NULL handle only
    # 512x512x160 needs several times the array
    for variant in range(5):
        rc, msg = call(variant, 512, 512, 160)
        assert rc == B.DIR_EINVAL and "scratch" in msg, msg
    # passive fits 11 M voxels, inverse-consistent 6.7 M: 320x320x100 (10.24 M) separates them
    assert call(B.DIR_PASSIVE, 320, 320, 100) == (B.DIR_EINVAL, "")
    rc, msg = call(B.DIR_INVERSE_CONSISTENT, 320, 320, 100)
    assert rc == B.DIR_EINVAL and "needs %d bytes" % need(B.DIR_INVERSE_CONSISTENT, 320 * 320 * 100, 8000) in msg, msg
