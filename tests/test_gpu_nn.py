"""Warm-start network kernels against the numpy reference (forward,
gradients, one Adam step), and the learned warm start against the plain
start of the static iteration on a small quasi-2D workload."""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)


def T():
    from paper_2602_08982_amd import tdslda
    tdslda.load_library()
    return tdslda


def data(C=8, B=3, H=6, W=5, seed=2):
    g = np.random.Generator(np.random.PCG64(seed))
    theta = (cnn.init_params(C, 3) + 0.05 * g.standard_normal(cnn.nparams(C))).astype(np.float32)
    x = g.standard_normal((B, 1, H, W)).astype(np.float32)
    Y = g.standard_normal((B, 2, H, W)).astype(np.float32)
    ymu = g.standard_normal(B).astype(np.float32)
    return theta, x, Y, ymu


def test_nn_forward_and_gradient_match_reference():
    t = T()
    C = 8
    theta, x, Y, ymu = data(C)
    net = t.Network(6, 5, C, 4, theta)
    try:
        maps, mu = net.forward(x)
        rm, rmu, _ = cnn.forward(theta.astype(float), x.astype(float), C)
        assert np.abs(maps - rm).max() / np.abs(rm).max() < 1e-5
        assert np.abs(mu - rmu).max() / np.abs(rmu).max() < 1e-5
        L, g = net.loss_grad(x, Y, ymu, 0.7)
        rL, rg = cnn.loss_and_grad(theta.astype(float), x.astype(float), Y.astype(float), ymu.astype(float), C, 0.7)
        assert abs(L - rL) / rL < 1e-5
        assert np.abs(g - rg).max() / np.abs(rg).max() < 1e-4
    finally:
        net.close()


def test_nn_adam_step_matches_reference():
    t = T()
    C = 8
    theta, x, Y, ymu = data(C)
    net = t.Network(6, 5, C, 4, theta)
    try:
        _, rg = cnn.loss_and_grad(theta.astype(float), x.astype(float), Y.astype(float), ymu.astype(float), C, 1.0)
        ref, _, _ = cnn.adam_step(theta.astype(float), rg, np.zeros_like(rg), np.zeros_like(rg), 1, 1e-3)
        net.train_step(x, Y, ymu, 1.0, 1e-3)
        th = net.params()
        assert np.abs(th - ref).max() < 2e-6
    finally:
        net.close()


def test_learned_warm_start_saves_iterations():
    """Trained on 48 method-generated solves of an 8x8x4 quasi-2D trap with
    random obstacles, the network's guess converges (no fallback) in fewer
    linear-mixing iterations than the uniform plain start on 8 held-out
    seeds; Broyden mixing (history 8) from the plain start also beats linear
    mixing (both are reported, with the warm start under Broyden mixing)."""
    from paper_2602_08982_amd import warmstart as WS
    cfg = dict(WS.Q2D, nx=8, ny=8, nz=4, omega=0.48, channels=16, maxit=400, coarse=6)
    res = WS.experiment(cfg, range(0, 48), range(10000, 10008), epochs=200)
    assert res["n_train"] >= 40
    assert res["fallbacks"] == 0
    assert res["warm_iters_mean"] < res["plain_iters_mean"], res
    # the non-learned accelerator the network is compared with
    assert res["plain_broyden_iters_mean"] < res["plain_iters_mean"], res
    # the coarse-lattice route (6x6 solve interpolated onto 8x8) converges
    assert res["coarse_start"]["fallbacks"] == 0, res["coarse_start"]
