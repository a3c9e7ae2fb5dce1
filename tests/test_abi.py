"""The C ABI library loads and exports every function include/cube.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cube.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cube_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for core in ("cube_create", "cube_init_ic", "cube_step", "cube_get_density", "cube_get_power", "cube_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1712_06121_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libcube.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(binding.EXPORTED) == declared()


def test_struct_layout_matches_header():
    from paper_1712_06121_amd.binding import CubeParams, CubeStateView
    assert ctypes.sizeof(CubeParams) == 8 * 4 + 8 * 8 + 8 + 8
    assert CubeParams.box.offset == 32 and CubeParams.seed.offset == 96
    assert ctypes.sizeof(CubeStateView) == 5 * 8 + 8 + 8 + 8


def test_footprint_is_host_arithmetic():
    """cube_footprint needs no device: it grows with the box and, at 2048^3 with 1-byte codes, is
    the resident state (180.1 GB: two particle buffers, coarse-cell arrays, the padded mesh) plus
    the two initial-condition displacement fields that do not fit in a particle buffer."""
    from paper_1712_06121_amd import footprint
    import synth
    c3 = synth.WORKLOADS["c3_pm2048"]
    fp = footprint(**c3)
    field = 2048 * 2048 * (1024 + 8) * 8
    resident = fp - 2 * field - 4 * (3 * 1024 * 1024 + 1)
    assert abs(resident / 180.1e9 - 1) < 1e-3
    sizes = [footprint(**dict(c3, np_side=n, nm_side=n, nc_side=n // 4)) for n in (64, 128, 256, 512)]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))


def test_counts_from_u8_is_host_only_and_matches_the_oracle():
    from paper_1712_06121_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libcube.so not built (run __graft_entry__.build())")
    import numpy as np
    from oracle import codec
    g = np.random.default_rng(5)
    counts = g.integers(0, 300, size=4096).astype(np.uint32)
    counts[[0, 17, 4095]] = [255, 1 << 20, 254]
    rho1, over = codec.counts_to_u8(counts)
    assert np.array_equal(binding.counts_from_u8(rho1, over), counts)
    with pytest.raises(binding.CubeError):
        binding.counts_from_u8(rho1, over[:-1])
