"""P15: the numpy reference of the warm-start network: backward pass
against central finite differences (FP64), the periodic 3x3 convolution
against a direct loop, and one Adam step against its definition."""
import numpy as np

from oracle import cnn


def test_conv3_matches_direct_loop():
    g = np.random.Generator(np.random.PCG64(1))
    x = g.standard_normal((2, 3, 5, 4))
    W = g.standard_normal((4, 3, 3, 3))
    b = g.standard_normal(4)
    y = cnn.conv3(x, W, b)
    ref = np.zeros_like(y)
    for n in range(2):
        for o in range(4):
            for i in range(5):
                for j in range(4):
                    s = b[o]
                    for c in range(3):
                        for di in range(3):
                            for dj in range(3):
                                s += W[o, c, di, dj] * x[n, c, (i + di - 1) % 5, (j + dj - 1) % 4]
                    ref[n, o, i, j] = s
    assert np.abs(y - ref).max() < 1e-12


def test_backward_matches_finite_differences():
    C = 4
    g = np.random.Generator(np.random.PCG64(2))
    theta = cnn.init_params(C, 3) + 0.05 * g.standard_normal(cnn.nparams(C))
    x = g.standard_normal((3, 1, 6, 5))
    Y = g.standard_normal((3, 2, 6, 5))
    ymu = g.standard_normal(3)
    L, grad = cnn.loss_and_grad(theta, x, Y, ymu, C, lam_mu=0.7)
    h = 1e-6
    idx = g.choice(theta.size, size=60, replace=False)
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (cnn.loss_and_grad(tp, x, Y, ymu, C, 0.7)[0] - cnn.loss_and_grad(tm, x, Y, ymu, C, 0.7)[0]) / (2 * h)
        assert abs(fd - grad[k]) < 1e-6 * max(1.0, abs(fd)), (k, fd, grad[k])


def test_adam_step_definition():
    th, gr = np.array([1.0, -2.0]), np.array([0.5, -0.25])
    m, v = np.zeros(2), np.zeros(2)
    th1, m1, v1 = cnn.adam_step(th, gr, m, v, 1, 0.1)
    # first step: bias-corrected m/sqrt(v) = sign(g)
    assert np.allclose(th1, th - 0.1 * np.sign(gr), atol=1e-7)
    assert np.allclose(m1, 0.1 * gr) and np.allclose(v1, 0.001 * gr * gr)
