"""Host-side checks of the synthetic inputs (no GPU): sizes, orientation,
load families."""
import numpy as np

from paper_2106_14189_amd import workloads as W


def test_box_mesh_orientation_and_faces():
    for elem in (W.T4, W.H8):
        m = W.box_mesh(4, 3, 5, 0.01, elem, jitter=0.05, seed=1)
        assert m.n_elems == 4 * 3 * 5 * (6 if elem == W.T4 else 1)
        assert m.n_nodes == 5 * 4 * 6
        if elem == W.T4:
            assert (W.signed_volume6(m.X, m.conn) > 0).all()
        np.testing.assert_allclose(m.X[m.bottom, 2], 0.0)
        np.testing.assert_allclose(m.X[m.top, 2], 0.05)


def test_config3_instances():
    b = W.config3(n_inst=24, n_steps=100)
    E = np.array([m.n_elems for m, _, _, _ in b])
    assert len(b) == 24 and E.min() >= 3000 and E.max() <= 260000
    for m, mat, ld, alpha in b:
        assert ld.t_ramp == -100.0 and alpha > 0
        assert len(ld.bc_node) == len(m.bottom) + len(m.top)
        amp = np.linalg.norm(ld.bc_target[len(m.bottom):], axis=1)
        assert np.all(amp >= 0.049 * m.height) and np.all(amp <= 0.201 * m.height)
        if m.ne == 4:
            assert (W.signed_volume6(m.X, m.conn) > 0).all()


def test_patch_family_windows_and_encoding():
    from paper_2106_14189_amd.warmstart import AMP_MAX, PatchFamily
    wl = W.config2(target_elems=6000)
    fam = PatchFamily(wl.mesh, seed=3)
    allp = np.concatenate(fam.patches)
    assert len(np.unique(allp)) == len(allp)                      # disjoint patches
    assert len(np.intersect1d(fam.fixed, allp)) == 0
    P = fam.sample(np.random.default_rng(0), 5)
    for p in P:
        t = fam.targets(p)
        assert np.abs(t[: len(fam.fixed)]).max() == 0.0
        assert np.linalg.norm(t, axis=1).max() <= AMP_MAX + 1e-15
    E = fam.encode(P)
    np.testing.assert_allclose(E[:, 3], P[:, 0])
    np.testing.assert_allclose(E[:, :3], P[:, :1] * P[:, 1:4])


def test_uniform_material_model_inputs():
    """TI/OT fibres are unit vectors, OT's second family is orthogonal to the
    first, ratios and C01 fall in their stated ranges."""
    rng = np.random.default_rng(3)
    E = rng.uniform(2000, 6000, 500)
    ot = W.uniform_material(500, E, 0.45, model=W.OT, rng=np.random.default_rng(1))
    np.testing.assert_allclose(np.linalg.norm(ot.fibre, axis=1), 1.0, rtol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(ot.fibre_b, axis=1), 1.0, rtol=1e-12)
    assert np.abs(np.sum(ot.fibre * ot.fibre_b, axis=1)).max() < 1e-12
    assert ot.eta_ratio.min() >= 2.0 and ot.eta_ratio.max() <= 10.0
    assert ot.eta_b_ratio.min() >= 2.0 and ot.eta_b_ratio.max() <= 10.0
    mr = W.uniform_material(500, E, 0.45, model=W.MR, rng=np.random.default_rng(2))
    c10 = E / (2 * 1.45) / 2
    r = mr.c01 / c10
    assert r.min() >= 0.2 and r.max() <= 1.0
    nh = W.uniform_material(500, E, 0.45)
    assert nh.fibre is None and nh.c01 is None
