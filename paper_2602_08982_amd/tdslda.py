"""ctypes binding of libtdslda (include/tdslda.h).  Argument marshalling only:
every step of the computation runs in the library's HIP kernels.

Host arrays are numpy float64 / complex128 in C order; states are
(n, 2, *grid) complex128 (component 0 = u, 1 = v).  Device arrays passed to
apply_hbdg are torch tensors (or raw integer device pointers).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdslda.so")

OK, EINVAL, ENOMEM, EDEVICE, EORDER, EUNSTABLE = 0, -1, -2, -3, -4, -5
MODE_3D, MODE_Q1D, MODE_Q2D = 3, 1, 2
FUNC_SLDA, FUNC_BDG, FUNC_ASLDA = 1, 2, 3
FP64, FP32_MIXED = 0, 1
AB3AM4, AB4AM5, AB5AM5 = 34, 45, 55


class Lattice(C.Structure):
    _fields_ = [("mode", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("lx_perp", C.c_double), ("ly_perp", C.c_double)]


class Functional(C.Structure):
    _fields_ = [("functional", C.c_int), ("A", C.c_double), ("B", C.c_double), ("C", C.c_double),
                ("inv_g_bdg", C.c_double), ("ec_reg", C.c_double), ("mu", C.c_double),
                ("temperature", C.c_double), ("mu_b", C.c_double)]


class Run(C.Structure):
    _fields_ = [("precision", C.c_int), ("integrator", C.c_int), ("dt", C.c_double),
                ("selfstart", C.c_int), ("taylor_order", C.c_int), ("tol_N", C.c_double),
                ("tol_E", C.c_double), ("hip_stream", C.c_void_p)]


class Static(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double), ("dy", C.c_double),
                ("dz", C.c_double), ("ec", C.c_double), ("mix", C.c_double), ("a_mu", C.c_double),
                ("N_req", C.c_double), ("tol", C.c_double), ("eF_ref", C.c_double), ("maxit", C.c_int),
                ("broyden", C.c_int), ("w0", C.c_double), ("q1d", C.c_int)]


class TdsldaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libtdslda status {status}: {msg}")
        self.status = status


_lib = None

_SIGS = {
    "tdslda_create": [C.POINTER(Lattice), C.POINTER(Functional), C.POINTER(Run), C.c_int64, C.POINTER(C.c_void_p)],
    "tdslda_destroy": [C.c_void_p],
    "tdslda_last_error": [C.c_void_p],
    "tdslda_memory_plan": [C.POINTER(Lattice), C.POINTER(Run), C.c_int64, C.POINTER(C.c_int64)],
    "tdslda_set_external": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int],
    "tdslda_set_regulator": [C.c_void_p, C.c_void_p],
    "tdslda_load_states": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_load_states_device": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_init_plane_waves": [C.c_void_p, C.c_int64, C.c_void_p, C.c_double, C.c_double],
    "tdslda_set_multiplicity": [C.c_void_p, C.c_int64, C.c_void_p],
    "tdslda_imprint_vortices": [C.c_void_p, C.c_int, C.c_void_p],
    "tdslda_set_fields": [C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_set_current_fields": [C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_densities": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_get_fields": [C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_densities_spin": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_apply_hbdg": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64],
    "tdslda_abm_step": [C.c_void_p, C.c_int64],
    "tdslda_energy": [C.c_void_p, C.c_void_p],
    "tdslda_check": [C.c_void_p, C.c_void_p],
    "tdslda_get_states": [C.c_void_p, C.c_void_p],
    "tdslda_info": [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "tdslda_save": [C.c_void_p, C.c_char_p],
    "tdslda_load": [C.c_void_p, C.c_char_p],
    "tdslda_set_profiling": [C.c_void_p, C.c_int],
    "tdslda_kernel_stats": [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "tdslda_kernel_name": [C.c_int],
    "tdslda_device_copy": [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p],
    "tdslda_device_read": [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p],
    "tdslda_abm_graph": [C.c_void_p, C.c_int64, C.c_void_p],
    "tdslda_autotune": [C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p],
    "tdslda_q1d_count": [C.POINTER(Lattice), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                         C.c_void_p, C.POINTER(C.c_int64)],
    "tdslda_static_map": [C.POINTER(Static), C.POINTER(Functional), C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)],
    "tdslda_static_solve": [C.POINTER(Static), C.POINTER(Functional), C.c_void_p, C.c_void_p, C.c_void_p,
                            C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_void_p],
    "tdslda_set_friction": [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double],
    "tdslda_interp2d": [C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int, C.c_double,
                        C.c_double, C.c_void_p],
    "tdslda_interp2d_noalloc": [C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int,
                                C.c_double, C.c_double, C.c_void_p, C.c_void_p],
    "tdslda_nn_nparams": [C.c_int],
    "tdslda_nn_create": [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)],
    "tdslda_nn_destroy": [C.c_void_p],
    "tdslda_nn_params": [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)],
    "tdslda_nn_set_params": [C.c_void_p, C.c_void_p],
    "tdslda_nn_forward": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
    "tdslda_nn_loss_grad": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_void_p,
                            C.c_void_p],
    "tdslda_nn_train_step": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_float,
                             C.c_void_p],
    "tdslda_q1d_load_static": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                               C.POINTER(C.c_int64)],
    "tdslda_q1d_count_spin": [C.POINTER(Lattice), C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_double, C.c_void_p, C.POINTER(C.c_int64)],
    "tdslda_q1d_load_static_spin": [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_double, C.POINTER(C.c_int64)],
}

EXPORTED = tuple(_SIGS)


def load_library(path=None):
    """Load libtdslda.so (raises if it is not built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("TDSLDA_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run python -m paper_2602_08982_amd.build")
    lib = C.CDLL(path)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = (C.c_char_p if name in ("tdslda_last_error", "tdslda_kernel_name")
                     else C.c_int64 if name == "tdslda_nn_nparams" else C.c_int)
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128_as_f64(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64)


def _dev_ptr(t):
    if isinstance(t, int):
        return C.c_void_p(t)
    return C.c_void_p(t.data_ptr())


def device_read(src, nbytes, sink, stream=None):
    """tdslda_device_read: streaming read of a device tensor (sink: a
    16-byte device tensor) on a HIP stream (integer handle; None = null)."""
    lib = load_library()
    st = lib.tdslda_device_read(_dev_ptr(src), int(nbytes), _dev_ptr(sink), C.c_void_p(stream or 0))
    if st != OK:
        raise TdsldaError(st, "device_read rejected the arguments")


def device_copy(dst, src, nbytes, stream=None):
    """tdslda_device_copy: streaming copy between device tensors (or raw
    device pointers) on a HIP stream (an integer handle; None = null)."""
    lib = load_library()
    st = lib.tdslda_device_copy(_dev_ptr(dst), _dev_ptr(src), int(nbytes), C.c_void_p(stream or 0))
    if st != OK:
        raise TdsldaError(st, "device_copy rejected the arguments")


def kernel_names():
    lib = load_library()
    out, k = [], 0
    while True:
        s = lib.tdslda_kernel_name(k)
        if s is None:
            return out
        out.append(s.decode())
        k += 1


def memory_plan(lattice, run, nstates):
    lib = load_library()
    b = C.c_int64()
    st = lib.tdslda_memory_plan(C.byref(lattice), C.byref(run), int(nstates), C.byref(b))
    if st != OK:
        raise TdsldaError(st, "memory_plan rejected the arguments")
    return b.value


class Context:
    """One libtdslda context (one stream)."""

    def __init__(self, lattice, functional, run, capacity):
        self.lib = load_library()
        self.lattice, self.functional, self.run = lattice, functional, run
        h = C.c_void_p()
        st = self.lib.tdslda_create(C.byref(lattice), C.byref(functional), C.byref(run), int(capacity), C.byref(h))
        if st != OK:
            raise TdsldaError(st, "tdslda_create failed (message on stderr)")
        self.h = h
        if lattice.mode == MODE_3D:
            self.grid = (lattice.nx, lattice.ny, lattice.nz)
        elif lattice.mode == MODE_Q2D:
            self.grid = (lattice.nx, lattice.ny)
        else:
            self.grid = (lattice.nz,)
        self.M = int(np.prod(self.grid))
        self.capacity = int(capacity)

    def _chk(self, st):
        if st != OK:
            msg = self.lib.tdslda_last_error(self.h)
            raise TdsldaError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.tdslda_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- set-up -----------------------------------------------------------
    def set_external(self, vext, freeze_regulator=True, dext=None):
        """V_ext (real) and optionally the external pairing potential
        Delta_ext (complex) on the lattice."""
        v = _f64(vext).ravel()
        d = None if dext is None else _c128_as_f64(np.asarray(dext).ravel())
        self._chk(self.lib.tdslda_set_external(self.h, _p(v), _p(d), int(freeze_regulator)))

    def set_regulator(self, lam):
        v = _f64(lam).ravel()
        self._chk(self.lib.tdslda_set_regulator(self.h, _p(v)))

    def load_states(self, phi, E, kperp2=None):
        phi = np.asarray(phi)
        n = phi.shape[0]
        uv = _c128_as_f64(phi.reshape(n, 2, self.M))
        e = _f64(E)
        k = None if kperp2 is None else _f64(kperp2)
        self._chk(self.lib.tdslda_load_states(self.h, n, _p(uv), _p(e), _p(k)))

    def load_states_device(self, tensor, n, E, kperp2=None):
        e = _f64(E)
        k = None if kperp2 is None else _f64(kperp2)
        self._chk(self.lib.tdslda_load_states_device(self.h, int(n), _dev_ptr(tensor), _p(e), _p(k)))

    def init_plane_waves(self, kidx, u0, delta0):
        k = np.ascontiguousarray(kidx, dtype=np.int32)
        self._chk(self.lib.tdslda_init_plane_waves(self.h, k.shape[0], _p(k), float(u0), float(delta0)))

    def set_multiplicity(self, mult):
        m = _f64(mult).ravel()
        self._chk(self.lib.tdslda_set_multiplicity(self.h, m.size, _p(m)))

    def imprint_vortices(self, vortices):
        v = _f64(vortices).reshape(-1, 3)
        self._chk(self.lib.tdslda_imprint_vortices(self.h, v.shape[0], _p(v)))

    def set_fields(self, U=None, delta=None):
        if U is None and delta is None:
            self._chk(self.lib.tdslda_set_fields(self.h, None, None))
            return
        u = _f64(U).ravel()
        d = _c128_as_f64(np.asarray(delta).ravel())
        self._chk(self.lib.tdslda_set_fields(self.h, _p(u), _p(d)))

    def set_current_fields(self, alpha=None, avec=None):
        """tdslda_set_current_fields: linear-mode alpha(r) and current
        potential of the general operator (3D: avec = (A_x, A_y, A_z) fields;
        quasi-1D: avec = A_z(z)); None keeps the functional's value."""
        a = None if alpha is None else _f64(alpha).ravel()
        z = None if avec is None else _f64(avec).ravel()
        self._chk(self.lib.tdslda_set_current_fields(self.h, _p(a), _p(z)))

    # --- evaluation ---------------------------------------------------------
    def densities(self):
        rho = np.empty(self.M)
        tau = np.empty(self.M)
        nu = np.empty(2 * self.M)
        j = np.empty(3 * self.M)
        self._chk(self.lib.tdslda_densities(self.h, _p(rho), _p(tau), _p(nu), _p(j)))
        g = self.grid
        return dict(rho=rho.reshape(g), tau=tau.reshape(g), nu=nu.view(np.complex128).reshape(g),
                    j=[j[i * self.M:(i + 1) * self.M].reshape(g) for i in range(3)])

    def densities_spin(self):
        """Spin-resolved densities of an ASLDA context: rho, tau, j as
        (spin a, spin b) pairs, nu."""
        rho = np.empty(2 * self.M)
        tau = np.empty(2 * self.M)
        nu = np.empty(2 * self.M)
        j = np.empty(6 * self.M)
        self._chk(self.lib.tdslda_densities_spin(self.h, _p(rho), _p(tau), _p(nu), _p(j)))
        g = self.grid
        sp = lambda a: (a[:self.M].reshape(g), a[self.M:].reshape(g))
        jj = j.reshape((2, 3) + g)
        return dict(rho=sp(rho), tau=sp(tau), nu=nu.view(np.complex128).reshape(g), j=(jj[0], jj[1]))

    def get_fields(self):
        ns = 2 if self.functional.functional == FUNC_ASLDA else 1
        U = np.empty(ns * self.M)
        d = np.empty(2 * self.M)
        self._chk(self.lib.tdslda_get_fields(self.h, _p(U), _p(d)))
        U = U.reshape(self.grid) if ns == 1 else (U[:self.M].reshape(self.grid), U[self.M:].reshape(self.grid))
        return U, d.view(np.complex128).reshape(self.grid)

    def apply_hbdg(self, x_dev, y_dev, n):
        self._chk(self.lib.tdslda_apply_hbdg(self.h, _dev_ptr(x_dev), _dev_ptr(y_dev), int(n)))

    def set_friction(self, alpha=0.0, beta=0.0, gamma=0.0, rho0=1.0, N_req=0.0):
        """Quantum-friction terms of the quasi-1D evolution (tdslda_set_friction)."""
        self._chk(self.lib.tdslda_set_friction(self.h, float(alpha), float(beta), float(gamma), float(rho0),
                                               float(N_req)))

    def abm_step(self, nsteps=1):
        self._chk(self.lib.tdslda_abm_step(self.h, int(nsteps)))

    def energy(self):
        out = np.empty(9)
        self._chk(self.lib.tdslda_energy(self.h, _p(out)))
        keys = ("kin", "pot", "pair", "curr", "potext", "total", "N", "EFG", "pairext")
        return dict(zip(keys, out.tolist()))

    def check(self):
        out = np.zeros(3)
        st = self.lib.tdslda_check(self.h, _p(out))
        return st, dict(dN=out[0], dE=out[1], norm=out[2])

    def get_states(self, n=None):
        nst, _, _ = self.info()
        out = np.empty((nst, 2) + self.grid, dtype=np.complex128)
        self._chk(self.lib.tdslda_get_states(self.h, _p(out.view(np.float64))))
        return out

    def info(self):
        n, s, t = C.c_int64(), C.c_int64(), C.c_double()
        self._chk(self.lib.tdslda_info(self.h, C.byref(n), C.byref(s), C.byref(t)))
        return n.value, s.value, t.value

    def save(self, path):
        self._chk(self.lib.tdslda_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._chk(self.lib.tdslda_load(self.h, os.fsencode(path)))

    def abm_graph(self, nsteps):
        """abm_step(nsteps) recorded as one HIP graph and launched once;
        returns (record + instantiate ms, launch-to-completion ms)."""
        ms = np.zeros(2)
        self._chk(self.lib.tdslda_abm_graph(self.h, int(nsteps), _p(ms)))
        return float(ms[0]), float(ms[1])

    def autotune(self):
        """Tune the launch shapes on the loaded states; returns a list of
        (workgroup size, median ms) per tuned kernel class."""
        n = C.c_int()
        ch = np.zeros(4, dtype=np.int32)
        ms = np.zeros(4)
        self._chk(self.lib.tdslda_autotune(self.h, C.byref(n), _p(ch), _p(ms)))
        return [(int(ch[i]), float(ms[i])) for i in range(n.value)]

    def q1d_load_static(self, kperp2, hfield, delta, ecut):
        """Load the static states (0 < E < ecut) of every quasi-1D problem;
        returns the number loaded."""
        kp = _f64(kperp2).ravel()
        hf = _f64(hfield).ravel()
        de = _f64(delta).ravel()
        n = C.c_int64()
        self._chk(self.lib.tdslda_q1d_load_static(self.h, kp.size, _p(kp), _p(hf), _p(de), float(ecut),
                                                  C.byref(n)))
        return n.value

    def q1d_load_static_spin(self, kperp2, hfield_a, hfield_b, delta, ecut):
        """Load both branches (|E| < ecut) of every spin-imbalanced quasi-1D
        problem; returns the number loaded."""
        kp = _f64(kperp2).ravel()
        ha = _f64(hfield_a).ravel()
        hb = _f64(hfield_b).ravel()
        de = _f64(delta).ravel()
        n = C.c_int64()
        self._chk(self.lib.tdslda_q1d_load_static_spin(self.h, kp.size, _p(kp), _p(ha), _p(hb), _p(de),
                                                       float(ecut), C.byref(n)))
        return n.value

    # --- profiling ----------------------------------------------------------
    def set_profiling(self, on=True):
        self._chk(self.lib.tdslda_set_profiling(self.h, int(on)))

    def kernel_stats(self):
        out = {}
        for k, name in enumerate(kernel_names()):
            n, ms = C.c_int64(), C.c_double()
            self._chk(self.lib.tdslda_kernel_stats(self.h, k, C.byref(n), C.byref(ms)))
            out[name] = (n.value, ms.value)
        return out


def q1d_count_spin(lattice, kperp2, hfield_a, hfield_b, delta, ecut):
    """Per-problem counts of both branches with |E| < ecut of the
    spin-imbalanced quasi-1D problems, and their total."""
    lib = load_library()
    kp = _f64(kperp2).ravel()
    ha = _f64(hfield_a).ravel()
    hb = _f64(hfield_b).ravel()
    de = _f64(delta).ravel()
    counts = np.zeros(kp.size, dtype=np.int32)
    tot = C.c_int64()
    st = lib.tdslda_q1d_count_spin(C.byref(lattice), kp.size, _p(kp), _p(ha), _p(hb), _p(de), float(ecut),
                                   _p(counts), C.byref(tot))
    if st != OK:
        raise TdsldaError(st, "tdslda_q1d_count_spin failed")
    return counts, tot.value


def q1d_count(lattice, kperp2, hfield, delta, ecut):
    """Per-problem counts of static states with 0 < E < ecut (eigenvalues
    only, on the device) and their total."""
    lib = load_library()
    kp = _f64(kperp2).ravel()
    hf = _f64(hfield).ravel()
    de = _f64(delta).ravel()
    counts = np.zeros(kp.size, dtype=np.int32)
    tot = C.c_int64()
    st = lib.tdslda_q1d_count(C.byref(lattice), kp.size, _p(kp), _p(hf), _p(de), float(ecut), _p(counts),
                              C.byref(tot))
    if st != OK:
        raise TdsldaError(st, "tdslda_q1d_count failed")
    return counts, tot.value


def static_params(nx, ny, nz, d=(1.0, 1.0, 1.0), ec=0.5 * np.pi ** 2, mix=0.5, a_mu=0.0, N_req=0.0, tol=1e-8,
                  eF_ref=0.5, maxit=500, broyden=0, w0=0.01, q1d=False):
    """q1d: the quasi-1D static geometry (nx lattice sites, ny plane waves
    along y, nz along z; fields of length nx)."""
    return Static(nx, ny, nz, d[0], d[1], d[2], ec, mix, a_mu, N_req, tol, eF_ref, maxit, broyden, w0, int(q1d))


def static_map(params, fun, vext, U, delta, mu):
    """One application of the static map K on the device: (U_out, delta_out,
    rho, nu, N)."""
    lib = load_library()
    shp = np.shape(vext)
    v, u, d = _f64(vext).ravel(), _f64(U).ravel(), _f64(delta).ravel()
    Uo, Do, rho, nu = (np.empty(v.size) for _ in range(4))
    N = C.c_double()
    st = lib.tdslda_static_map(C.byref(params), C.byref(fun), _p(v), _p(u), _p(d), float(mu), _p(Uo), _p(Do),
                               _p(rho), _p(nu), C.byref(N))
    if st != OK:
        raise TdsldaError(st, "tdslda_static_map failed")
    return Uo.reshape(shp), Do.reshape(shp), rho.reshape(shp), nu.reshape(shp), N.value


def static_solve(params, fun, vext, U, delta, mu):
    """Self-consistent iteration on the device from (U, delta, mu).  Returns
    (U, delta, mu, iterations, converged, history[iterations][4])."""
    lib = load_library()
    shp = np.shape(vext)
    v = _f64(vext).ravel()
    u, d = _f64(U).ravel().copy(), _f64(delta).ravel().copy()
    m = C.c_double(float(mu))
    it, ok = C.c_int(), C.c_int()
    hist = np.zeros((params.maxit, 4))
    st = lib.tdslda_static_solve(C.byref(params), C.byref(fun), _p(v), _p(u), _p(d), C.byref(m), C.byref(it),
                                 C.byref(ok), _p(hist))
    if st != OK:
        raise TdsldaError(st, "tdslda_static_solve failed")
    return u.reshape(shp), d.reshape(shp), m.value, it.value, bool(ok.value), hist[:it.value]


def interp2d(f, d, shape2, d2):
    """Fourier interpolation of a real x-y field onto another lattice of the
    same box (tdslda_interp2d); d, d2 = (dx, dy) spacings."""
    lib = load_library()
    f = _f64(f)
    nx, ny = f.shape
    nx2, ny2 = shape2
    out = np.empty(nx2 * ny2)
    st = lib.tdslda_interp2d(nx, ny, float(d[0]), float(d[1]), _p(f.ravel()), nx2, ny2, float(d2[0]), float(d2[1]),
                             _p(out))
    if st != OK:
        raise TdsldaError(st, "tdslda_interp2d failed")
    return out.reshape(nx2, ny2)


def interp2d_noalloc(f_dev, d, out_dev, d2, stream=None):
    """tdslda_interp2d_noalloc: the same interpolation between device
    tensors (FP64, shapes (nx, ny) and (nx2, ny2)), queued on `stream`
    (a hipStream_t handle, None = null stream); no device allocation."""
    lib = load_library()
    for t in (f_dev, out_dev):
        if t.dim() != 2 or not t.is_cuda or t.dtype.itemsize != 8 or not t.is_floating_point() or \
                not t.is_contiguous():
            raise ValueError("interp2d_noalloc takes contiguous 2D float64 device tensors")
    nx, ny = f_dev.shape
    nx2, ny2 = out_dev.shape
    st = lib.tdslda_interp2d_noalloc(nx, ny, float(d[0]), float(d[1]), _dev_ptr(f_dev), nx2, ny2, float(d2[0]),
                                     float(d2[1]), _dev_ptr(out_dev), C.c_void_p(stream or 0))
    if st != OK:
        raise TdsldaError(st, "tdslda_interp2d_noalloc failed")


class Network:
    """The warm-start network (tdslda_nn_*): float32 host arrays in, out."""

    def __init__(self, H, W, channels, batch_max, theta0):
        self.lib = load_library()
        self.H, self.W, self.C, self.batch_max = H, W, channels, batch_max
        self.P = int(self.lib.tdslda_nn_nparams(channels))
        th = np.ascontiguousarray(theta0, dtype=np.float32).ravel()
        if th.size != self.P:
            raise ValueError(f"theta0 has {th.size} values, the network {self.P}")
        hp = C.c_void_p()
        st = self.lib.tdslda_nn_create(H, W, channels, batch_max, th.ctypes.data_as(C.c_void_p), C.byref(hp))
        if st != OK:
            raise TdsldaError(st, "tdslda_nn_create failed")
        self.h = hp

    def close(self):
        if getattr(self, "h", None):
            self.lib.tdslda_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st, what):
        if st != OK:
            raise TdsldaError(st, what)

    def params(self):
        out = np.empty(self.P, dtype=np.float32)
        self._chk(self.lib.tdslda_nn_params(self.h, out.ctypes.data_as(C.c_void_p), None), "tdslda_nn_params")
        return out

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32).ravel()
        self._chk(self.lib.tdslda_nn_set_params(self.h, th.ctypes.data_as(C.c_void_p)), "tdslda_nn_set_params")

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        B = x.shape[0]
        maps = np.empty((B, 2, self.H, self.W), dtype=np.float32)
        mu = np.empty(B, dtype=np.float32)
        self._chk(self.lib.tdslda_nn_forward(self.h, B, x.ctypes.data_as(C.c_void_p), maps.ctypes.data_as(C.c_void_p),
                                             mu.ctypes.data_as(C.c_void_p)), "tdslda_nn_forward")
        return maps, mu

    def loss_grad(self, x, Y, ymu, lam_mu=1.0):
        x, Y, ymu = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, Y, ymu))
        loss = np.zeros(1, dtype=np.float32)
        grad = np.empty(self.P, dtype=np.float32)
        self._chk(self.lib.tdslda_nn_loss_grad(self.h, x.shape[0], x.ctypes.data_as(C.c_void_p),
                                               Y.ctypes.data_as(C.c_void_p), ymu.ctypes.data_as(C.c_void_p),
                                               float(lam_mu), loss.ctypes.data_as(C.c_void_p),
                                               grad.ctypes.data_as(C.c_void_p)), "tdslda_nn_loss_grad")
        return float(loss[0]), grad

    def train_step(self, x, Y, ymu, lam_mu, lr):
        x, Y, ymu = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, Y, ymu))
        loss = np.zeros(1, dtype=np.float32)
        self._chk(self.lib.tdslda_nn_train_step(self.h, x.shape[0], x.ctypes.data_as(C.c_void_p),
                                                Y.ctypes.data_as(C.c_void_p), ymu.ctypes.data_as(C.c_void_p),
                                                float(lam_mu), float(lr), loss.ctypes.data_as(C.c_void_p)),
                  "tdslda_nn_train_step")
        return float(loss[0])


def lattice_3d(n, d=1.0):
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    return Lattice(MODE_3D, nx, ny, nz, dx, dy, dz, 0.0, 0.0)


def lattice_q1d(nz, dz, lx, ly):
    return Lattice(MODE_Q1D, 1, 1, nz, 1.0, 1.0, dz, lx, ly)


def lattice_q2d(nx, ny, nz, d=(1.0, 1.0, 1.0)):
    """Quasi-2D: nx x ny x-y lattice, nz plane waves along z (L_z = nz dz)."""
    dx, dy, dz = (d, d, d) if np.isscalar(d) else d
    return Lattice(MODE_Q2D, nx, ny, nz, dx, dy, dz, 0.0, 0.0)


def functional_slda(mu, ec_reg, A=1.0, B=None, C_=-11.11, temperature=0.0):
    """Unitary-gas SLDA at p = 0: A = 1 (the A_sigma = 1 option) or the
    general functional with A = 1.094; B defaults to the ASLDA formula
    evaluated with A_a = A_b = A, B = 2^(2/3) 0.357 - A."""
    if B is None:
        B = 2.0 ** (2.0 / 3.0) * 0.357 - A
    return Functional(FUNC_SLDA, A, B, C_, 0.0, ec_reg, mu, temperature)


def functional_aslda(mu_a, mu_b, ec_reg, temperature=0.0):
    """Spin-imbalanced ASLDA (A_a(p), A_b(p), B(p), C = -11.11 of the local
    polarisation) with the chemical potentials of both spins."""
    return Functional(FUNC_ASLDA, 0.0, 0.0, -11.11, 0.0, ec_reg, mu_a, temperature, mu_b)


def functional_bdg(mu, ec_reg, a_s, temperature=0.0):
    return Functional(FUNC_BDG, 1.0, 0.0, 0.0, 1.0 / (4.0 * np.pi * a_s), ec_reg, mu, temperature)


def run_config(precision=FP64, integrator=AB4AM5, dt=0.005, selfstart=1, taylor_order=5,
               tol_N=0.0, tol_E=0.0, stream=None):
    return Run(precision, integrator, dt, selfstart, taylor_order, tol_N, tol_E, stream)
