"""GPU checks of the boundary calls around the solves: the tile autotuner's persistent cache
(bl_autotune writes an entry; a later call takes the stored height without timing), recycle
storage carved by bl_recycle_init (every Session uses it), and the RGen-L(R) refresh where
rank(J W) is below both s and p with p > 64 (the null-space fill of the GSVD selection)."""
import numpy as np
import pytest

import synth
from oracle import problem, recycle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08264_amd import bilevel
    return bilevel


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def test_autotune_cache_roundtrip(B, tmp_path):
    wl = synth.custom("t", 64, "tv", 4, blur_radius=2, blur_sigma=1.5, seed=91)
    inst = synth.instance(wl)
    P = B.problem_from(wl)
    path = str(tmp_path / "tiles.txt")
    xh = dev(inst["xstar"].ravel())
    with B.Session(P, s_max=4, v_cap=0) as S:
        try:
            rows, us = S.autotune_tiles(P, inst["theta0"], xh, 4, iters=12, cache_path=path)
            assert rows in (8, 16, 32) and all(u > 0.0 for u in us)
            assert B.bl_tile_rows(P) == rows
            lines = [l.split() for l in open(path) if not l.startswith("#")]
            assert len(lines) == 1
            # key: reg radius n_filters filter_size prec log2 n; then the height and the timings
            assert [int(v) for v in lines[0][:7]] == [0, 2, 0, 0, 0, 12, rows]
            assert np.allclose([float(v) for v in lines[0][7:]], us, rtol=1e-3, atol=1e-3)
            B.bl_tile_rows_set(P, 0)
            # stored entry: no timing (zeros), same height
            rows2, us2 = S.autotune_tiles(P, inst["theta0"], xh, 4, iters=12, cache_path=path)
            assert rows2 == rows and us2 == (0.0, 0.0, 0.0) and B.bl_tile_rows(P) == rows
            # a second class is added to the same file, the first entry kept
            P2 = B.problem_from(synth.custom("u", 48, "tv", 4, blur_radius=1, blur_sigma=1.0, seed=92))
            x2 = dev(synth.instance(synth.custom("u", 48, "tv", 4, blur_radius=1, blur_sigma=1.0, seed=92))
                     ["xstar"].ravel())
            with B.Session(P2, s_max=4, v_cap=0) as S2:
                S2.autotune_tiles(P2, inst["theta0"], x2, 4, iters=12, cache_path=path)
            assert len([l for l in open(path) if not l.startswith("#")]) == 2
            B.bl_tile_rows_set(P, 0)
            B.bl_tile_rows_set(P2, 0)
            assert B.bl_tile_cache_load(path) == 2 and B.bl_tile_rows(P) == rows
        finally:
            B.bl_tile_rows_set(P, 0)


def test_recycle_storage_views(B):
    """The binding's Recycle tensors are views of the one buffer bl_recycle_init carved."""
    wl = synth.custom("t", 40, "tv", 5, width=24, blur_radius=1, blur_sigma=1.0, seed=93)
    P = B.problem_from(wl)
    rec = B.Recycle(wl.n, 5, 7, DEV, P)
    assert rec.nbytes() == B.lib.bl_recycle_bytes(B.C.byref(P), 5, 7)
    assert rec.U.data_ptr() == rec.rs.U and rec.Cm.data_ptr() == rec.rs.C and rec.Z.data_ptr() == rec.rs.Z
    assert rec.mu.data_ptr() == rec.rs.mu and rec.V.data_ptr() == rec.rs.V
    assert tuple(rec.U.shape) == (5, wl.n) and tuple(rec.V.shape) == (7, wl.n) and rec.mu.numel() == 5
    assert all(t.data_ptr() % 256 == 0 for t in (rec.U, rec.Cm, rec.Z, rec.mu, rec.V))
    assert float(rec.buf.abs().max()) == 0.0


def test_refresh_fill_when_rank_g_below_p_above_64(B):
    """Filters with p = 3 (1 + 5^2) = 78 at x_hat = 0: phi'(K x_hat) = 0 and x_hat = 0 make
    J W = 0, so every slot of RGen-L(R) is filled by Ritz-S vectors of H on null(G) = range(W)
    (t = 84 > p).  The GPU selection matches the oracle's subspace; mu = 0 and Z = 0."""
    wl = synth.custom("f", 24, "filters", 6, n_filters=3, filter_size=5, rect_min=2, rect_max=6, seed=94)
    assert wl.p == 78
    inst = synth.instance(wl)
    prob = problem.make_problem(wl, inst["xstar"], inst["e"])
    th = inst["theta0"]
    xh = np.zeros(prob.n)
    hvp = lambda v: prob.hvp(xh, th, v)
    V = synth.unit_noise((prob.n, 84), 95)   # a well-conditioned basis: no column is dropped
    ref = recycle.refresh(hvp, lambda v: prob.jac_apply(xh, th, v), None, V, s=6)
    assert ref["rank_G"] == 0 and ref["t"] == 84
    with B.Session(B.problem_from(wl), s_max=6, v_cap=84) as S:
        S.V[:84] = dev(V.T)
        S.rs.v_cur = 84
        st = S.refresh(th, dev(xh), s=6)
        assert S.rs.s_cur == 6 and st.t == 84 and st.iters == 0   # stats.iters: rank of G
        U = host(S.U[:6]).T
        assert recycle.principal_angles(U, ref["U"]).max() <= 1e-8
        assert float(S.mu[:6].abs().max()) == 0.0 and float(S.Z[:6].abs().max()) == 0.0
        C = host(S.Cm[:6]).T
        HU = np.stack([hvp(U[:, j]) for j in range(6)], axis=1)
        assert np.linalg.norm(HU - C) <= 1e-11 * np.linalg.norm(C)
