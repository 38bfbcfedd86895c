"""Learned warm start on a small ellipsoid (about 6000 TI tetrahedra): the
network is trained on the GPU from steady states of the plain relaxation, and
its prediction must reach a relative displacement error of 1e-3 against the
converged plain solution in fewer steps and less device and wall time
(inference included) than the plain solve from rest with the best ramp
length of a sweep that includes applying the load at once."""
import sys

import pytest

from paper_2106_14189_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_warm_start_beats_cold_start():
    assert torch.cuda.is_available()
    from paper_2106_14189_amd import warmstart
    wl = W.config2(target_elems=6000)
    r = warmstart.experiment(wl.mesh, wl.material, wl.alpha, n_train=512, n_test=8, seed=5, relax_steps=6000,
                             t_ramp=0.4, hidden=512, epochs=150, batch=64, lr=1e-3, log=say)
    for k, v in r.items():
        say(f"  {k}: {v}")
    assert r["all_reached"]
    assert r["held_out_residual_max"] < 1e-5
    assert r["train_loss_first_last"][1] < 0.05 * r["train_loss_first_last"][0]
    assert r["cold_ramp_s"] is not None
    assert r["warm_steps_median"] < r["cold_steps_median"]
    assert r["warm_device_ms_median"] < r["cold_device_ms_median"]
    assert r["warm_wall_ms_median"] < r["cold_wall_ms_median"]
