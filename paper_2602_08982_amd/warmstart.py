"""Learned warm start of the static solve (host-side orchestration only: the
solves run in libtdslda's device solver, the network in its kernels).

Workload: a quasi-2D trapped gas on an nx x ny x-y lattice with nz plane
waves along z, V_ext = 1/2 omega^2 (x^2 + y^2) + 1-4 Gaussian obstacles
(amplitudes U(0.5, 3) eF_ref, widths U(2, 8) sites of a 64-site box scaled
to the lattice, uniform centres), fixed particle number N_req = N of the
obstacle-free trap at mu = 1.  The plain start is the uniform state at the
reference Fermi momentum k_F = 1 (eF_ref = 1/2); the warm start is the
network's prediction of (U, Delta, mu) from V_ext.  Both are iterated by the
same mixing to r < tol (linear mixing, and the modified Broyden mixing as
the non-learned accelerator to compare with); when the warm start does not
converge the plain start is used (and counted).  The non-learned starts of
Sec. 5.2 run beside it: the coarse-lattice start (refining lattice
resolution) and the symmetry-release start (quasi-1D first).
"""
import time

import numpy as np

from . import tdslda as T

EF_REF = 0.5
XI_UFG = 0.4     # mu / eF of the uniform unitary gas (plain start)
DELTA_UFG = 0.5  # Delta / eF of the uniform unitary gas (plain start)

Q2D = dict(nx=16, ny=16, nz=8, omega=0.24, mix=0.5, a_mu=0.5, tol=1e-8, maxit=400, channels=32, broyden=8,
           w0=0.01, coarse=12)


def vext(cfg, seed, nx=None, ny=None):
    """V_ext on the nx x ny lattice of the target box (default: the target
    lattice itself, spacing 1; a coarser lattice has spacing L / nx), at the
    centred coordinates x = (i - nx/2) d."""
    import synth
    L_x, L_y = cfg["nx"], cfg["ny"]
    nx = L_x if nx is None else nx
    ny = L_y if ny is None else ny
    x = (np.arange(nx) - nx // 2) * (L_x / nx)
    y = (np.arange(ny) - ny // 2) * (L_y / ny)
    X, Y = np.meshgrid(x, y, indexing="ij")
    v = 0.5 * cfg["omega"] ** 2 * (X ** 2 + Y ** 2)
    amp, wid, cen = synth.obstacles(seed, float(L_x))
    s = L_x / 64.0
    for a, w, (cx, cy) in zip(amp, wid, cen):
        v = v + EF_REF * a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * (w * s) ** 2))
    return v


def plain_start(cfg, fun):
    U = np.full((cfg["nx"], cfg["ny"]), fun.B * EF_REF)
    D = np.full((cfg["nx"], cfg["ny"]), DELTA_UFG * EF_REF)
    return U, D, XI_UFG * EF_REF


def params(cfg, N_req=0.0, a_mu=None, broyden=0):
    """Solver parameters.  A coarse lattice (spacing cfg["d"] > 1) keeps the
    target lattice's regulator cut-off (pi^2/2): the coarse solve is a guess
    for the target problem, and its own lattice cut-off would leave the
    regulator undefined where V_ext - mu exceeds it."""
    d = cfg.get("d", 1.0)
    return T.static_params(cfg["nx"], cfg["ny"], cfg["nz"], d=(d, d, 1.0), ec=0.5 * np.pi ** 2, mix=cfg["mix"],
                           a_mu=cfg["a_mu"] if a_mu is None else a_mu, N_req=N_req, tol=cfg["tol"],
                           eF_ref=EF_REF, maxit=cfg["maxit"], broyden=broyden, w0=cfg.get("w0", 0.01))


def required_n(cfg, fun):
    """N of the obstacle-free trap at mu = 1 (fixed-mu solve)."""
    nx, ny = cfg["nx"], cfg["ny"]
    x = np.arange(nx) - nx // 2
    y = np.arange(ny) - ny // 2
    X, Y = np.meshgrid(x, y, indexing="ij")
    v = 0.5 * cfg["omega"] ** 2 * (X ** 2 + Y ** 2)
    U0, D0, _ = plain_start(cfg, fun)
    U, D, mu, it, ok, hist = T.static_solve(params(cfg, a_mu=0.0), fun, v, U0, D0, 1.0)
    if not ok:
        raise RuntimeError("reference trap did not converge")
    _, _, _, _, N = T.static_map(params(cfg), fun, v, U, D, mu)
    return N


def solve(cfg, fun, N_req, v, start, broyden=0):
    U0, D0, mu0 = start
    t0 = time.perf_counter()
    U, D, mu, it, ok, hist = T.static_solve(params(cfg, N_req, broyden=broyden), fun, v, U0, D0, mu0)
    return dict(U=U, D=D, mu=mu, iters=it, converged=ok, seconds=time.perf_counter() - t0)


def coarse_start(cfg, fun, N_req, seed, nxc, broyden=0):
    """Sec. 5.2, refining lattice resolution: solve on an nxc x nxc lattice of
    the same box (spacing nx / nxc), then interpolate (U, Delta) onto the
    target lattice (tdslda_interp2d); mu carries over.  Returns (start,
    coarse result)."""
    d = cfg["nx"] / nxc
    cc = dict(cfg, nx=nxc, ny=nxc, d=d)
    vc = vext(cfg, seed, nxc, nxc)
    U0, D0, mu0 = plain_start(cc, fun)
    t0 = time.perf_counter()
    U, D, mu, it, ok, hist = T.static_solve(params(cc, N_req, broyden=broyden), fun, vc, U0, D0, mu0)
    res = dict(iters=it, converged=ok, seconds=time.perf_counter() - t0)
    shape = (cfg["nx"], cfg["ny"])
    Uf = T.interp2d(U, (d, d), shape, (1.0, 1.0))
    Df = T.interp2d(D, (d, d), shape, (1.0, 1.0))
    return (Uf, Df, mu), res


def release_start(cfg, fun, N_req, broyden=0):
    """Sec. 5.2, releasing symmetry constraints: first the quasi-1D problem
    with the trap along y switched off (omega_y = 0; the obstacles, which
    break the symmetry, are left out): an nx-site x lattice with ny plane
    waves along y (the target's L_y) and nz along z, V = 1/2 omega^2 x^2, the
    same N_req, from the plain start; then its (U(x), Delta(x)) repeated
    along y and its mu start the quasi-2D solve.  The first stage does not
    depend on the obstacles.  Returns (start, quasi-1D result)."""
    nx, ny = cfg["nx"], cfg["ny"]
    x = (np.arange(nx) - nx // 2) * 1.0
    v1 = 0.5 * cfg["omega"] ** 2 * x ** 2
    p = T.static_params(nx, ny, cfg["nz"], d=(1.0, 1.0, 1.0), ec=0.5 * np.pi ** 2, mix=cfg["mix"],
                        a_mu=cfg["a_mu"], N_req=N_req, tol=cfg["tol"], eF_ref=EF_REF, maxit=cfg["maxit"],
                        broyden=broyden, w0=cfg.get("w0", 0.01), q1d=True)
    U0 = np.full(nx, fun.B * EF_REF)
    D0 = np.full(nx, DELTA_UFG * EF_REF)
    t0 = time.perf_counter()
    U, D, mu, it, ok, hist = T.static_solve(p, fun, v1, U0, D0, XI_UFG * EF_REF)
    res = dict(iters=it, converged=ok, seconds=time.perf_counter() - t0)
    start = (np.repeat(U[:, None], ny, axis=1), np.repeat(D[:, None], ny, axis=1), mu)
    return start, res


class WarmStart:
    """Normalisation + network; fit() trains on method-generated solves."""

    def __init__(self, cfg, seed=0, batch_max=64):
        self.cfg = cfg
        C = cfg["channels"]
        g = np.random.Generator(np.random.PCG64(seed))
        parts = []
        for name, s in _shapes(C):
            if name.startswith("b"):
                parts.append(np.zeros(s))
            else:
                fan_in = int(np.prod(s[1:])) if len(s) > 1 else s[0]
                parts.append(g.standard_normal(s) * np.sqrt(2.0 / fan_in))
        theta0 = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
        self.net = T.Network(cfg["nx"], cfg["ny"], C, batch_max, theta0)
        self.batch_max = batch_max
        self.xs = 1.0

    def _x(self, vs):
        return (np.asarray(vs)[:, None] / self.xs).astype(np.float32)

    def fit(self, V, U, D, mu, epochs=300, lr=2e-3, lam_mu=1.0, seed=1):
        V = np.asarray(V)
        self.xs = float(np.abs(V).max())
        X = self._x(V)
        Y = np.stack([np.asarray(U) / EF_REF, np.asarray(D) / EF_REF], axis=1).astype(np.float32)
        ym = (np.asarray(mu) / EF_REF).astype(np.float32)
        g = np.random.Generator(np.random.PCG64(seed))
        n = X.shape[0]
        B = min(self.batch_max, n)
        losses = []
        steps = 0
        for ep in range(epochs):
            perm = g.permutation(n)
            rate = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
            for b0 in range(0, n - B + 1, B):
                idx = perm[b0:b0 + B]
                losses.append(self.net.train_step(X[idx], Y[idx], ym[idx], lam_mu, rate))
                steps += 1
        return dict(steps=steps, final_loss=float(np.mean(losses[-10:])), first_loss=float(losses[0]))

    def predict(self, V):
        maps, mu = self.net.forward(self._x(V))
        return maps[:, 0].astype(float) * EF_REF, maps[:, 1].astype(float) * EF_REF, mu.astype(float) * EF_REF

    def close(self):
        self.net.close()


def _shapes(C):
    return [("W1", (C, 1, 3, 3)), ("b1", (C,)), ("W2", (C, C, 3, 3)), ("b2", (C,)),
            ("W3", (C, C, 3, 3)), ("b3", (C,)), ("Wm", (2, C)), ("bm", (2,)), ("wmu", (C,)), ("bmu", (1,))]


def experiment(cfg, train_seeds, test_seeds, epochs=300, log=None):
    """Train on solves of train_seeds, then compare iterations to r < tol
    from the plain and the warm start on test_seeds."""
    fun = T.functional_slda(1.0, 0.5 * np.pi ** 2)
    N_req = required_n(cfg, fun)
    t0 = time.perf_counter()
    V, U, D, MU, it_train = [], [], [], [], []
    nb = cfg.get("broyden", 0)
    for i, s in enumerate(train_seeds):
        if log and i and i % 10 == 0:
            log(f"training solves: {i} of {len(train_seeds)} ({time.perf_counter() - t0:.0f} s)")
        v = vext(cfg, s)
        # the training targets are fixed points of K; the Broyden iteration
        # reaches the same ones in fewer maps
        r = solve(cfg, fun, N_req, v, plain_start(cfg, fun), broyden=nb)
        if not r["converged"]:
            continue
        V.append(v)
        U.append(r["U"])
        D.append(r["D"])
        MU.append(r["mu"])
        it_train.append(r["iters"])
    t_data = time.perf_counter() - t0
    if log:
        log(f"training set: {len(V)} solves in {t_data:.1f} s, mean {np.mean(it_train):.1f} iterations")
    ws = WarmStart(cfg)
    t0 = time.perf_counter()
    fit = ws.fit(V, U, D, MU, epochs=epochs)
    t_fit = time.perf_counter() - t0
    if log:
        log(f"fit: {fit['steps']} Adam steps in {t_fit:.1f} s, loss {fit['first_loss']:.3g} -> {fit['final_loss']:.3g}")
    # iterations to r < tol from the plain and the warm start, with linear
    # mixing and (nb > 0) with Broyden mixing; a warm start that does not
    # converge falls back to the plain start and is charged maxit extra
    its = {k: [] for k in ("plain", "warm", "plain_broyden", "warm_broyden")}
    fallbacks, plain_s, plain_it = 0, 0.0, 0
    # the mixings compared: linear (unless cfg["linear"] is False) and Broyden
    mixings = ([("", 0)] if cfg.get("linear", True) else []) + ([("_broyden", nb)] if nb else [])
    coarse = {k: [] for k in ("coarse", "fine", "coarse_broyden", "fine_broyden")}
    coarse.update(fallbacks=0, coarse_s=0.0, coarse_it=0)
    # releasing symmetry constraints: the quasi-1D stage is the same for
    # every seed; it is solved once per mixing and charged to every seed
    rel = {k: [] for k in ("fine", "fine_broyden")}
    rel_stage = {}
    if cfg.get("release", True):
        for suffix, b in mixings:
            rel_stage[suffix] = release_start(cfg, fun, N_req, broyden=b)
    rel_fallbacks = 0
    for i, s in enumerate(test_seeds):
        if log and i and i % 5 == 0:
            log(f"held-out seeds: {i} of {len(test_seeds)}")
        v = vext(cfg, s)
        Uw, Dw, muw = ws.predict(v[None])
        warm = (Uw[0], Dw[0], float(muw[0]))
        for suffix, b in mixings:
            p = solve(cfg, fun, N_req, v, plain_start(cfg, fun), broyden=b)
            w = solve(cfg, fun, N_req, v, warm, broyden=b)
            plain_s += p["seconds"]
            plain_it += p["iters"]
            its["plain" + suffix].append(p["iters"])
            if w["converged"]:
                its["warm" + suffix].append(w["iters"])
            else:
                fallbacks += 1
                its["warm" + suffix].append(p["iters"] + cfg["maxit"])
        nxc = cfg.get("coarse", 0)
        for suffix, b in (mixings if nxc else ()):
            start, cres = coarse_start(cfg, fun, N_req, s, nxc, broyden=b)
            f = solve(cfg, fun, N_req, v, start, broyden=b)
            coarse["coarse" + suffix].append(cres["iters"])
            coarse["fine" + suffix].append(f["iters"] if f["converged"] else f["iters"] + cfg["maxit"])
            coarse["fallbacks"] += 0 if (f["converged"] and cres["converged"]) else 1
            coarse["coarse_s"] += cres["seconds"]
            coarse["coarse_it"] += cres["iters"]
        for suffix, b in (mixings if rel_stage else ()):
            start, sres = rel_stage[suffix]
            f = solve(cfg, fun, N_req, v, start, broyden=b)
            rel["fine" + suffix].append(f["iters"] if f["converged"] else f["iters"] + cfg["maxit"])
            rel_fallbacks += 0 if (f["converged"] and sres["converged"]) else 1
    ws.close()
    out = dict(lattice=[cfg["nx"], cfg["ny"], cfg["nz"]], n_train=len(V), n_test=len(test_seeds),
               train_data_seconds=t_data, fit_seconds=t_fit, fit=fit, fallbacks=fallbacks,
               seconds_per_iteration=plain_s / max(1, plain_it), N_req=N_req, broyden=nb)
    if its["plain"]:
        out.update(plain_iters_mean=float(np.mean(its["plain"])), warm_iters_mean=float(np.mean(its["warm"])),
                   plain_iters=its["plain"], warm_iters=its["warm"])
    if coarse["coarse"] or coarse["coarse_broyden"]:
        # cost of a coarse iteration in target-lattice iterations, measured
        ratio = (coarse["coarse_s"] / max(1, coarse["coarse_it"])) / out["seconds_per_iteration"]
        cres = dict(lattice=[cfg["coarse"], cfg["coarse"], cfg["nz"]], cost_ratio=ratio, fallbacks=coarse["fallbacks"])
        for suffix in ("", "_broyden"):
            if coarse["coarse" + suffix]:
                c, f = np.mean(coarse["coarse" + suffix]), np.mean(coarse["fine" + suffix])
                cres["linear" if not suffix else "broyden"] = dict(coarse_iters_mean=float(c), fine_iters_mean=float(f),
                                                                   target_equivalent=float(c * ratio + f))
        out["coarse_start"] = cres
    if rel_stage:
        # cost of a quasi-1D iteration in target-lattice iterations, measured
        s1 = sum(r["seconds"] for _, r in rel_stage.values())
        i1 = sum(r["iters"] for _, r in rel_stage.values())
        ratio = (s1 / max(1, i1)) / out["seconds_per_iteration"]
        rres = dict(stage1="quasi-1D: x lattice, plane waves along y and z, omega_y = 0, no obstacles, same N",
                    cost_ratio=ratio, fallbacks=rel_fallbacks)
        for suffix in ("", "_broyden"):
            if rel["fine" + suffix]:
                c1 = rel_stage[suffix][1]["iters"]
                f = float(np.mean(rel["fine" + suffix]))
                rres["linear" if not suffix else "broyden"] = dict(
                    q1d_iters=int(c1), q2d_iters_mean=f, target_equivalent=float(c1 * ratio + f),
                    target_equivalent_once=float(f + c1 * ratio / max(1, len(test_seeds))))
        out["symmetry_release_start"] = rres
    if its["plain_broyden"]:
        out.update(plain_broyden_iters_mean=float(np.mean(its["plain_broyden"])),
                   warm_broyden_iters_mean=float(np.mean(its["warm_broyden"])),
                   plain_broyden_iters=its["plain_broyden"], warm_broyden_iters=its["warm_broyden"])
    return out
