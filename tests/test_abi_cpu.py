"""Host-only checks of the C ABI: the library loads, exports every declared entry point,
and answers the calls that need no GPU (sizes, parameter counts, status strings,
argument validation before any launch)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bilevel.h")
LIB = os.path.join(ROOT, "paper_2412_08264_amd", "libbilevel_hip.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:bl_status|size_t|int|const char\*)\s+(bl_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    from paper_2412_08264_amd import bilevel as B
    names = declared_symbols()
    assert len(names) >= 14
    raw = C.CDLL(LIB)
    for name in names:
        assert hasattr(raw, name), name
    assert set(names) == set(B.EXPORTED)


def test_sizes_and_counts():
    from paper_2412_08264_amd import bilevel as B
    import synth
    P = B.problem_from(synth.WORKLOADS["tv256"])
    assert B.bl_num_params(P) == 2
    nb = B.bl_workspace_bytes(P, 20, 64)
    assert nb > 65536 * 8 * 2 * 84
    Pf = B.problem_from(synth.WORKLOADS["foe512"])
    assert B.bl_num_params(Pf) == 400
    assert B.bl_workspace_bytes(Pf, 30, 64) > B.bl_workspace_bytes(Pf, 10, 16)
    assert B.bl_workspace_bytes(P, 65, 10) == 0          # s_max above the compiled limit
    assert B.bl_workspace_bytes(P, 20, 300) == 0         # refresh width above the limit


def test_status_strings_and_null_context():
    from paper_2412_08264_amd import bilevel as B
    assert B.lib.bl_status_string(B.BL_E_INDEFINITE).decode().startswith("non-positive")
    assert B.lib.bl_status_string(99).decode() == "unknown status"
    P = B.bl_problem(8, 8, 1, 1.0, B.BL_REG_TV, 0, 0, 0.0, 0, 0)
    opts = B.bl_solve_opts(0, 1e-10, 0.0, 10, 1, 0, 0)
    st = B.bl_stats()
    th = (C.c_double * 2)(0.0, 0.0)
    # null context is rejected before anything touches a device
    assert B.lib.bl_hessian_solve(None, C.byref(P), th, None, None, None, None, C.byref(opts), None, 0,
                                  C.byref(st)) == B.BL_E_ARG
    assert B.lib.bl_destroy(None) == B.BL_E_ARG
    assert B.lib.bl_hessian_solve_rminres(None, C.byref(P), th, None, None, None, None, C.byref(opts), None, 0,
                                          C.byref(st)) == B.BL_E_ARG
    ro = B.bl_recycle_opts(4, 1e-8, 0)
    assert B.lib.bl_recycle_update(None, C.byref(P), th, None, None, C.byref(ro), None, 0, C.byref(st)) == B.BL_E_ARG


def test_selection_codes_match_header():
    """The binding's selection names map to the codes bl_select declares, in Table 2's order."""
    from paper_2412_08264_amd import bilevel as B
    text = open(HEADER).read()
    codes = {m.group(1).lower().replace("_", "-"): int(m.group(2))
             for m in re.finditer(r"BL_SEL_(\w+)\s*=\s*(\d+)", text)}
    assert codes == B.SELECTIONS
    assert len(set(codes.values())) == 15


def test_engine_sizes():
    from paper_2412_08264_amd import bilevel as B
    import synth
    P = B.problem_from(synth.WORKLOADS["tv256"])
    lib = B.lib
    s0 = lib.bl_engine_slot_bytes(C.byref(P), 0)
    s20 = lib.bl_engine_slot_bytes(C.byref(P), 20)
    assert s0 >= 4 * 8 * 65536 and s20 > s0
    assert lib.bl_engine_slot_bytes(C.byref(P), 65) == 0
    Pf = B.problem_from(synth.WORKLOADS["foe512"])
    # filter slots hold the phi'' maps: 8 filters x (two FP64 + one FP32) maps
    assert lib.bl_engine_slot_bytes(C.byref(Pf), 0) >= (4 + 8 * 2.5) * 8 * 512 * 512
    assert lib.bl_engine_workspace_bytes(0, 1024) == 0 and lib.bl_engine_workspace_bytes(65, 1024) == 0
    assert lib.bl_engine_workspace_bytes(64, 10 ** 6) >= 10 ** 6
    arr = (B.bl_problem * 2)(P, P)
    sv = (C.c_int * 2)(20, 0)
    assert lib.bl_batched_workspace_bytes(2, arr, sv) >= s20 + s0
    assert lib.bl_batched_workspace_bytes(0, arr, sv) == 0


def test_engine_argument_checks_without_gpu():
    from paper_2412_08264_amd import bilevel as B
    P = B.bl_problem(8, 8, 1, 1.0, B.BL_REG_TV, 0, 0, 0.0, 0, 0)
    eng = C.c_void_p()
    assert B.lib.bl_engine_create(None, 2, None, 0, C.byref(eng)) == B.BL_E_ARG
    assert B.lib.bl_engine_destroy(None) == B.BL_E_ARG
    nd = C.c_int()
    assert B.lib.bl_engine_step(None, 1, 1, None, C.byref(nd)) == B.BL_E_ARG


def test_tile_height_table_without_gpu():
    """Default tile height: the tallest of 32/16/8 rows that gives the image >= 256 tiles of 32
    columns, else 8; table entries override it per operator class and size class (log2 n)."""
    from paper_2412_08264_amd import bilevel as B
    mk = lambda h, w, reg=B.BL_REG_TV, prec=0: B.bl_problem(h, w, 4, 2.5, reg, 8 if reg else 0, 7 if reg else 0,
                                                            0.0, 0, prec)
    tiles = lambda h, w, rows: -(-w // 32) * -(-h // rows)
    for h, w in [(256, 256), (512, 512), (384, 384), (128, 128), (1024, 1024), (64, 64), (3, 2000)]:
        want = next((r for r in (32, 16) if tiles(h, w, r) >= 256), 8)
        assert B.bl_tile_rows(mk(h, w)) == want, (h, w)
    P, Pq = mk(256, 256), mk(200, 300)          # n = 65536 and 60000: size classes 16 and 15
    Pf = mk(256, 256, B.BL_REG_FILTERS)
    B.bl_tile_rows_set(P, 32)
    try:
        assert B.bl_tile_rows(P) == 32 and B.bl_tile_rows(mk(300, 250)) == 32   # same size class
        assert B.bl_tile_rows(Pq) == B.bl_tile_rows(mk(200, 300, prec=1)) == 8  # other classes
        assert B.bl_tile_rows(Pf) == 8
        with pytest.raises(B.BLError):
            B.bl_tile_rows_set(P, 24)
        with pytest.raises(B.BLError):
            B.bl_tile_rows_set(B.bl_problem(1, 1, 0, 1.0, 0, 0, 0, 0.0, 0, 0), 8)
    finally:
        B.bl_tile_rows_set(P, 0)
    assert B.bl_tile_rows(P) == 8
    assert B.lib.bl_tile_rows(None) == 0
    nul = C.c_int()
    assert B.lib.bl_autotune(None, C.byref(P), None, None, 0, 10, None, None, 0, C.byref(nul), None) == B.BL_E_ARG
    assert B.lib.bl_autotune_workspace_bytes(C.byref(P), 20) >= B.bl_workspace_bytes(P, 20, 0) + (2 + 3 * 20) * 8 * 65536
    assert B.lib.bl_autotune_workspace_bytes(C.byref(P), 65) == 0


def test_tile_cache_file_without_gpu(tmp_path):
    """bl_tile_cache_load: entries of the autotuner's cache file go into the tile table by
    operator class and size class; a malformed or missing file is refused and loads nothing."""
    from paper_2412_08264_amd import bilevel as B
    P = B.bl_problem(256, 256, 4, 2.5, B.BL_REG_TV, 0, 0, 0.0, 0, 0)          # TV r=4 FP64, log2 n = 16
    Pf = B.bl_problem(512, 512, 5, 3.0, B.BL_REG_FILTERS, 8, 7, 1e-6, 0, 1)   # filters 8x7x7 mixed, 18
    good = tmp_path / "tiles.txt"
    good.write_text("# reg radius n_filters filter_size prec log2n rows us8 us16 us32\n"
                    "0 4 0 0 0 16 32 30.0 28.0 25.0\n"
                    "1 5 8 7 1 18 16 900.0 850.0 870.0\n")
    try:
        assert B.bl_tile_cache_load(str(good)) == 2
        assert B.bl_tile_rows(P) == 32 and B.bl_tile_rows(Pf) == 16
        B.bl_tile_rows_set(P, 0)
        B.bl_tile_rows_set(Pf, 0)
        bad = tmp_path / "bad.txt"
        bad.write_text("0 4 0 0 0 16 32 30.0 28.0 25.0\n1 5 8 7 1 18 12 1 2 3\n")   # 12 rows: invalid
        with pytest.raises(B.BLError):
            B.bl_tile_cache_load(str(bad))
        assert B.bl_tile_rows(P) == 8                # nothing from the bad file was loaded
        with pytest.raises(B.BLError):
            B.bl_tile_cache_load(str(tmp_path / "missing.txt"))
        assert B.lib.bl_tile_cache_load(None, None) == B.BL_E_ARG
    finally:
        B.bl_tile_rows_set(P, 0)
        B.bl_tile_rows_set(Pf, 0)


def test_recycle_storage_layout_without_gpu():
    """bl_recycle_bytes / bl_recycle_init: U, C, Z (n x s_max), mu (s_max), V (n x v_cap), in that
    order, each on a 256-byte boundary, carved from one caller buffer (host only: the addresses
    are never dereferenced, so a fake aligned base serves)."""
    from paper_2412_08264_amd import bilevel as B
    al = lambda b: -(-b // 256) * 256
    P = B.bl_problem(96, 80, 2, 1.5, B.BL_REG_TV, 0, 0, 0.0, 0, 0)
    n, s, v = 96 * 80, 10, 50
    want = 3 * al(8 * n * s) + al(8 * s) + al(8 * n * v) + al(16 * v)
    assert B.lib.bl_recycle_bytes(C.byref(P), s, v) == want
    assert B.lib.bl_recycle_bytes(C.byref(P), 65, 0) == 0 and B.lib.bl_recycle_bytes(C.byref(P), 20, 237) == 0
    assert B.lib.bl_recycle_bytes(None, 4, 4) == 0
    assert B.lib.bl_recycle_bytes(C.byref(P), 0, 0) == 256     # empty storage: still a valid shape
    base = 1 << 40
    rs = B.bl_recycle()
    assert B.lib.bl_recycle_init(C.byref(P), s, v, C.c_void_p(base), want, C.byref(rs)) == B.BL_OK
    assert (rs.U, rs.C, rs.Z, rs.mu, rs.V) == (base, base + al(8 * n * s), base + 2 * al(8 * n * s),
                                               base + 3 * al(8 * n * s), base + 3 * al(8 * n * s) + al(8 * s))
    assert rs.lz == rs.V + al(8 * n * v)
    assert (rs.s_max, rs.s_cur, rs.v_cap, rs.v_cur, rs.v_lz) == (s, 0, v, 0, 0)
    assert B.lib.bl_recycle_init(C.byref(P), s, v, C.c_void_p(base), want - 1, C.byref(rs)) == B.BL_E_WORKSPACE
    assert B.lib.bl_recycle_init(C.byref(P), s, v, C.c_void_p(base + 8), want, C.byref(rs)) == B.BL_E_WORKSPACE
    assert B.lib.bl_recycle_init(C.byref(P), 65, v, C.c_void_p(base), want, C.byref(rs)) == B.BL_E_SHAPE
    assert B.lib.bl_recycle_init(C.byref(P), s, v, None, want, C.byref(rs)) == B.BL_E_ARG
    rs0 = B.bl_recycle()
    assert B.lib.bl_recycle_init(C.byref(P), 4, 0, C.c_void_p(base), want, C.byref(rs0)) == B.BL_OK
    assert rs0.V is None and rs0.lz is None and rs0.v_cap == 0
