"""Several load cases per launch (djtled_step_multi) on the GPU.

Each case must reproduce a separate djtled_step run bit for bit (same
chunks, same summation order, same arithmetic); one case is also checked
against the FP64 oracle to the FP32 full-run tolerance (1e-4 relative
max-norm displacement error).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2106_14189_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2106_14189_amd import solver
    return solver


def _setup(S, elem, model, prec="fp32", n=9, seed=5, variant=-1):
    mesh = W.cube_mesh(n, 0.1 / n, elem, jitter=0.05, seed=seed, permute=True)
    rng = np.random.default_rng(seed)
    E = rng.uniform(2000.0, 6000.0, mesh.n_elems)
    mat = W.uniform_material(mesh.n_elems, E, 0.45, 1000.0, model=model, rng=rng)
    sv = S.Solver(mesh.X, mesh.conn, mat.E, mat.nu, model=model, eta_ratio=mat.eta_ratio, fibre=mat.fibre,
                  eta_b_ratio=mat.eta_b_ratio, fibre_b=mat.fibre_b, c01=mat.c01, precision=prec, alpha=37.0,
                  variant=variant)
    return mesh, mat, sv


def _cases(mesh, sv, strains, t_ramp):
    """One compression case per strain, plus a lateral shear of the top face on odd cases."""
    out = []
    for i, e in enumerate(strains):
        ld = W.compression_loads(mesh, e, W.RAMP_SMOOTH, t_ramp)
        tgt = ld.bc_target.copy()
        if i % 2:
            top = np.isin(ld.bc_node, mesh.top)
            tgt[top, 0] = 0.3 * e * mesh.height
        out.append((ld, sv.loadset(ld.bc_node, np.where(np.isin(ld.bc_node, mesh.top), 7, ld.bc_mask) if i % 2
                                   else ld.bc_mask, tgt, ld.ramp, ld.t_ramp)))
    return out


@pytest.mark.parametrize("elem", [W.T4, W.H8])
@pytest.mark.parametrize("model", [W.NH, W.TI])
@pytest.mark.parametrize("k", [2, 3, 8])
def test_multi_equals_single_runs(S, elem, model, k):
    mesh, mat, sv = _setup(S, elem, model)
    dt = sv.info()["dt"]
    n = 300
    cases = _cases(mesh, sv, [-0.05 - 0.02 * i for i in range(k)], n * dt)
    say(f"multi elem={elem} model={model} k={k}: {sv.info()['n_elems']} elements")
    U, UP = sv.zeros_multi(k), sv.zeros_multi(k)
    # two launches (splitting is neutral for single runs too)
    st, step, res, ec = sv.step_multi(U, UP, 120, [ls for _, ls in cases])
    assert st.code == 0 and st.steps_done == 120 and ec == -1
    st, step, res, ec = sv.step_multi(U, UP, n - 120, [ls for _, ls in cases], step0=step)
    assert st.code == 0 and step == n
    torch.cuda.synchronize()
    for i, (_, ls) in enumerate(cases):
        u, up = sv.zeros(), sv.zeros()
        st1, _ = sv.step(u, up, n, ls)
        assert st1.code == 0
        assert torch.equal(U[i], u) and torch.equal(UP[i], up), f"case {i} differs from its single run"
    assert float(U.abs().max()) > 0


def test_multi_against_oracle(S):
    """Case 1 of a three-case FP32 run against the FP64 oracle."""
    mesh, mat, sv = _setup(S, W.T4, W.NH, n=8, seed=3)
    ora = oracle.Oracle(mesh.X, mesh.conn, mat.E, mat.nu, rho=1000.0)
    dt = 0.9 * ora.dt_crit
    assert abs(sv.info()["dt"] - dt) <= 1e-15 * dt
    n = 400
    cases = _cases(mesh, sv, [-0.1, -0.15, -0.2], n * dt)
    U, UP = sv.zeros_multi(3), sv.zeros_multi(3)
    st, _, _, _ = sv.step_multi(U, UP, n, [ls for _, ls in cases])
    assert st.code == 0
    ld = cases[2][0]
    uo, upo = np.zeros((ora.n_nodes, 3)), np.zeros((ora.n_nodes, 3))
    rc, done, _ = ora.run(uo, upo, n, dt, 37.0, ld.bc_node, ld.bc_mask, ld.bc_target, ramp=ld.ramp, t_ramp=ld.t_ramp)
    assert rc == 0 and done == n
    err = np.abs(U[2].double().cpu().numpy() - uo).max() / np.abs(uo).max()
    say(f"multi case 2 vs oracle: rel max displacement error {err:.3e}")
    assert err <= 1e-4


def test_multi_relax_all_cases_converge(S):
    mesh, mat, sv = _setup(S, W.H8, W.NH, n=6, seed=2)
    dt = sv.info()["dt"]
    cases = _cases(mesh, sv, [-0.05, -0.1], 200 * dt)
    U, UP = sv.zeros_multi(2), sv.zeros_multi(2)
    st, step, res, ec = sv.step_multi(U, UP, 200000, [ls for _, ls in cases], relax=True, tol=1e-4, check_every=50)
    say(f"multi relax: code {st.code} steps {st.steps_done} residuals {res}")
    assert st.code == 1 and np.all(res <= 1e-4) and st.residual == res.max()
    # each case alone converges no later than the pair
    for i, (_, ls) in enumerate(cases):
        u, up = sv.zeros(), sv.zeros()
        st1, _ = sv.step(u, up, 200000, ls, relax=True, tol=1e-4, check_every=50)
        assert st1.code == 1 and st1.steps_done <= st.steps_done


def test_multi_error_names_the_case(S):
    mesh = W.cube_mesh(2, 0.01, W.T4, jitter=0.0)
    sv = S.Solver(mesh.X, mesh.conn, 3000.0, 0.45, precision="fp32", alpha=0.0)
    top = mesh.top
    mild = sv.loadset(top, np.full(len(top), 4), np.tile([0, 0, -0.0001], (len(top), 1)), ramp=W.RAMP_NONE)
    crush = sv.loadset(top, np.full(len(top), 4), np.tile([0, 0, -0.05], (len(top), 1)), ramp=W.RAMP_NONE)
    U, UP = sv.zeros_multi(2), sv.zeros_multi(2)
    st, step, res, ec = sv.step_multi(U, UP, 50, [mild, crush], raise_on_error=False)
    assert st.code == -3 and ec == 1 and st.steps_done == 1 and st.error_step == 1
    # both cases stop at the last completed step
    assert torch.all(U[1, top, 2] == -0.05) and torch.all(U[0, top, 2] == -0.0001)
    assert torch.count_nonzero(UP) == 0


def test_multi_argument_errors(S):
    from paper_2106_14189_amd import _lib as L
    mesh, mat, sv = _setup(S, W.T4, W.NH, n=3)
    dt = sv.info()["dt"]
    ld = W.compression_loads(mesh, -0.1, W.RAMP_SMOOTH, 10 * dt)
    a = sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, ld.t_ramp)
    b = sv.loadset(ld.bc_node, ld.bc_mask, ld.bc_target, ld.ramp, 2 * ld.t_ramp)
    U, UP = sv.zeros_multi(2), sv.zeros_multi(2)
    with pytest.raises(L.DJError, match="ramp"):
        sv.step_multi(U, UP, 5, [a, b])
    U9, UP9 = sv.zeros_multi(9), sv.zeros_multi(9)
    with pytest.raises(L.DJError):
        sv.step_multi(U9, UP9, 5, None)
    # no loads at all: a free body at rest stays at rest
    st, _, _, _ = sv.step_multi(U, UP, 5, None)
    assert st.code == 0 and torch.count_nonzero(U) == 0
    # several cases are built for FP32 contexts
    s64 = S.Solver(mesh.X, mesh.conn, 3000.0, 0.45, precision="fp64")
    with pytest.raises(L.DJError, match="UNSUPPORTED"):
        s64.step_multi(s64.zeros_multi(2), s64.zeros_multi(2), 5, None)
