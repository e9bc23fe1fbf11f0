"""The C-ABI library without a GPU: it loads, exports every function that
include/mra.h declares, and its host-side argument checks and size queries
behave as documented (no kernel is launched by any call here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mra.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    from paper_1604_08159_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libmra.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("mra_transform", "collocation_rhs", "krylov_step", "solve_batch", "mra_solve_init",
              "mra_solve_read", "mra_solve_footprint", "mra_status_str"):
        assert n in names, n


def test_every_declared_symbol_is_exported(lib):
    from paper_1604_08159_amd import _lib
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mra.h but not exported"
        assert n in _lib.EXPORTS, f"{n} has no binding"


def test_status_strings_and_version(lib):
    assert lib.mra_abi_version() == 1
    assert lib.mra_status_str(0).decode() == "ok"
    assert "argument" in lib.mra_status_str(1).decode()
    assert lib.mra_status_str(99).decode() == "unknown status"


def _grid(J, p, eps=1e-3, j0=None):
    from paper_1604_08159_amd._lib import GridDesc
    import math
    return GridDesc(J, (2 if p == 2 else 3) if j0 is None else j0, p, 1, 2 * math.pi, eps)


def test_size_queries_and_argument_checks(lib):
    n = C.c_size_t()
    assert lib.mra_solve_footprint(C.byref(_grid(9, 2)), 2, 20, C.byref(n)) == 0
    fp_mixed = n.value
    assert lib.mra_solve_footprint(C.byref(_grid(9, 2)), 0, 20, C.byref(n)) == 0
    assert n.value > fp_mixed                                   # FP64 fields are larger
    # the arena holds at least the Krylov basis (m+1) x N^2 FP64
    assert fp_mixed > 21 * 512 * 512 * 8
    assert lib.mra_solve_footprint(C.byref(_grid(12, 2)), 2, 20, C.byref(n)) == 2     # J too large
    assert lib.mra_solve_footprint(C.byref(_grid(2, 2)), 2, 20, C.byref(n)) == 2      # J <= j0
    assert lib.mra_solve_footprint(C.byref(_grid(9, 4)), 2, 20, C.byref(n)) == 2      # p unsupported
    assert lib.mra_solve_footprint(C.byref(_grid(9, 2, j0=3)), 2, 20, C.byref(n)) == 2  # wrong j0
    assert lib.mra_solve_footprint(C.byref(_grid(9, 2)), 2, 48, C.byref(n)) == 2     # m too large
    assert lib.mra_solve_footprint(C.byref(_grid(9, 2, eps=-1.0)), 2, 20, C.byref(n)) == 1
    assert lib.mra_transform_ws_bytes(C.byref(_grid(9, 3)), 0, C.byref(n)) == 0 and n.value > 0
    assert lib.mra_rhs_ws_bytes(C.byref(_grid(9, 3)), 1, C.byref(n)) == 0 and n.value > 0
    # null pointers are rejected before anything is launched
    assert lib.mra_transform(C.byref(_grid(5, 2)), 0, 1, None, None, None, None, None, None, None, 0, None) == 1
    assert lib.krylov_step(None, 1, None) == 1
    assert lib.solve_batch(None, 0, None, None) == 1
    assert lib.mra_solve_destroy(None) == 1
    assert lib.mra_solve_track(None, 2, (C.c_double * 4)(), None) == 1
    assert lib.mra_scalar_init(None, C.byref(_grid(6, 2)), 10, 0.01, 0.0, 1, None, None, 0, None,
                               C.byref(C.c_void_p())) == 1
    assert lib.mra_solve_set_integrator(None, 1, 0.5, 2, None) == 1
    assert lib.mra_solve_set_jacobian(None, 1) == 1
    assert lib.mra_scalar_set_condensation(None, 1.0, None) == 1


def test_tile_table_host_logic():
    """mra_tune_set_tile / mra_tune_get_tile on the host: defaults, the
    precisions that share bulk storage, the accepted edges, and that the
    footprint of a new solve follows the table (its tile-count array)."""
    import paper_1604_08159_amd as m
    from paper_1604_08159_amd import autotune as at
    assert m.tune_get_tile(9, 2, m.MRA_MIXED) == 32
    assert m.tune_get_tile(9, 3, m.MRA_FP64) == 16
    assert m.tune_get_tile(3, 2, m.MRA_MIXED) == 8
    g = m.grid_desc(9, 2, 1e-4)
    f32 = m.solve_footprint(g, m.MRA_MIXED, 20)
    try:
        m.tune_set_tile(9, 2, m.MRA_MIXED, 16)
        assert m.tune_get_tile(9, 2, m.MRA_MIXED) == 16 and m.tune_get_tile(9, 2, m.MRA_FP32) == 16
        assert m.tune_get_tile(9, 2, m.MRA_FP64) == 32
        assert m.solve_footprint(g, m.MRA_MIXED, 20) > f32          # four times the tile counts
    finally:
        m.tune_set_tile(9, 2, m.MRA_MIXED, 0)
    assert m.tune_get_tile(9, 2, m.MRA_MIXED) == 32
    for bad in [(9, 3, m.MRA_FP64, 32), (4, 2, m.MRA_MIXED, 32), (9, 2, m.MRA_MIXED, 12), (2, 2, m.MRA_MIXED, 8),
                (12, 2, m.MRA_MIXED, 16), (9, 4, m.MRA_MIXED, 16), (9, 2, 3, 16)]:
        with pytest.raises(m.MraError) as e:
            m.tune_set_tile(*bad)
        assert e.value.status == 1
    assert at.valid_tiles(9, 3, m.MRA_FP64) == (8, 16)
    assert at.valid_tiles(4, 2, m.MRA_MIXED) == (8, 16)
    assert at.valid_tiles(11, 3, m.MRA_MIXED) == (8, 16, 32)
    assert at.parse_entry_key(at.entry_key(10, 3, 2)) == (10, 3, 2)


def test_noalloc_transform_host_checks(lib):
    """mra_transform_noalloc on the host: every grid up to J = 10 fits its
    5 MiB per-device workspace whatever the tile table holds, a larger grid
    is refused with MRA_E_SIZE and null arrays with MRA_E_ARG, both before
    anything touches the GPU."""
    import paper_1604_08159_amd as m
    n = C.c_size_t()
    limit = 5 << 20
    try:
        for J in range(3, 11):
            for p in (2, 3):
                if J <= (2 if p == 2 else 3):
                    continue
                for prec in (0, 1, 2):
                    for tile in (0, 8, 16, 32):
                        if tile and (tile > (1 << J) or (prec == 0 and p == 3 and tile == 32)):
                            continue
                        m.tune_set_tile(J, p, prec, tile)
                        assert lib.mra_transform_ws_bytes(C.byref(_grid(J, p)), prec, C.byref(n)) == 0
                        assert n.value <= limit, (J, p, prec, tile, n.value)
                        m.tune_set_tile(J, p, prec, 0)
    finally:
        for J in range(3, 11):
            for p in (2, 3):
                for prec in (0, 2):
                    if J > (2 if p == 2 else 3):
                        m.tune_set_tile(J, p, prec, 0)
    buf = C.c_void_p(0x1000)     # never dereferenced: the size check comes first
    assert lib.mra_transform_noalloc(C.byref(_grid(11, 2)), 0, 1, buf, buf, None, None, None, None, None) == 2
    assert lib.mra_transform_noalloc(C.byref(_grid(11, 3)), 2, 2, buf, buf, buf, None, buf, buf, None) == 2
    assert lib.mra_transform_noalloc(C.byref(_grid(6, 2)), 0, 1, None, None, None, None, None, None, None) == 1
    assert lib.mra_transform_noalloc(C.byref(_grid(6, 2)), 0, 7, buf, buf, None, None, None, None, None) == 1


def test_capacity_footprint_and_checks(lib):
    """The arena of a solve sized for `capacity` active nodes: the active-length
    arrays and the Krylov basis shrink with it, the node-indexed fields do
    not; 0 means N^2; out-of-range capacities are refused before anything is
    allocated or launched."""
    n, full, zero = C.c_size_t(), C.c_size_t(), C.c_size_t()
    g = _grid(9, 2)
    nf = 512 * 512
    assert lib.mra_solve_footprint(C.byref(g), 2, 20, C.byref(full)) == 0
    assert lib.mra_solve_footprint_cap(C.byref(g), 2, 20, 0, C.byref(zero)) == 0
    assert zero.value == full.value
    assert lib.mra_solve_footprint_cap(C.byref(g), 2, 20, nf, C.byref(n)) == 0 and n.value == full.value
    sizes = []
    for cap in (16, 4096, 20000, 65536, nf // 2):
        assert lib.mra_solve_footprint_cap(C.byref(g), 2, 20, cap, C.byref(n)) == 0
        sizes.append(n.value)
    assert sizes == sorted(sizes) and sizes[-1] < full.value
    # per active node: FP64 value, two int32 indices, FP64 w, m + 1 FP64 basis
    # entries and the adapted evaluation's level byte (within the 256-byte
    # alignment of each array)
    per_node = 8 + 4 + 4 + 8 + 21 * 8 + 1
    assert abs((sizes[3] - sizes[2]) - per_node * (65536 - 20000)) <= 16 * 256
    # a small capacity takes the residual's FP64 prolongation out of the basis
    assert lib.mra_solve_footprint_cap(C.byref(g), 0, 20, 4096, C.byref(n)) == 0
    assert lib.mra_solve_footprint_cap(C.byref(g), 2, 20, 15, C.byref(n)) == 2       # below the coarsest mesh
    assert lib.mra_solve_footprint_cap(C.byref(g), 2, 20, nf + 1, C.byref(n)) == 2   # above N^2
    assert lib.mra_solve_footprint_cap(C.byref(g), 2, 20, -5, C.byref(n)) == 2
    assert lib.mra_solve_capacity(None, C.byref(C.c_int64()), C.byref(C.c_int64()), C.byref(C.c_int32()),
                                  None) == 1
    assert lib.mra_solve_migrate(None, 4096, None, 0, None) == 1
    assert lib.mra_solve_init_cap(C.byref(g), None, 2, 20, 0.01, None, 4096, None, 0, None,
                                  C.byref(C.c_void_p()), None) != 0
    assert lib.mra_status_str(7) == b"active set exceeds the solve's capacity"


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library every entry of the binding raises: there is
    no CPU path behind it."""
    import paper_1604_08159_amd as m
    from paper_1604_08159_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libmra.so"))
    monkeypatch.setattr(m, "_LIB", None)
    with pytest.raises(ImportError):
        _lib.load()
    with pytest.raises(ImportError):
        m.lib()
    with pytest.raises(ImportError):
        m.solve_footprint(m.grid_desc(7, 2, 1e-4), m.MRA_FP64, 10)
