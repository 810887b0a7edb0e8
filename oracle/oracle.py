"""ctypes front end of the FP64 C oracle (``hho_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every method maps to one
C routine; the arithmetic lives in C, written from the paper:
  * eq. HHO1 / HHO2, eq. rec_a / rec_e, eq. stab (Sec. 3.3) for the operator,
  * eq. ex_solve (Sec. 4.2) for the condensed explicit stage,
  * eq. ERK for the Butcher tableaux, the energy of Sec. 5.1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hho_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Butcher tableaux of eq. ERK: (A, b, c) for s = 2, 3, 4
ERK_TABLEAUX = {
    2: (np.array([[0, 0], [0.5, 0]]), np.array([0.0, 1.0]), np.array([0.0, 0.5])),
    3: (np.array([[0, 0, 0], [0.5, 0, 0], [-1.0, 2.0, 0]]), np.array([1 / 6, 2 / 3, 1 / 6]),
        np.array([0.0, 0.5, 1.0])),
    4: (np.array([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]]),
        np.array([1 / 6, 1 / 3, 1 / 3, 1 / 6]), np.array([0.0, 0.5, 0.5, 1.0])),
}


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP) into oracle/liboracle.so: -O3 for the x86-64-v3
    level (AVX2, FMA), which every host that runs it supports; -march=native is not used because
    the library is built on one machine and run on another."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build_oracle())
        P, I, D, V = C.c_void_p, C.c_int, C.c_double, None
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        sig = {
            "orc_create": (P, [I, dp, I, ip, ip, up, dp, dp, dp, I, D, D, I]),
            "orc_destroy": (V, [P]),
            "orc_ndof": (I, [P]), "orc_nfaces": (I, [P]), "orc_nface_dofs": (I, [P]),
            "orc_offsets": (V, [P, ip]), "orc_face_offsets": (V, [P, ip]),
            "orc_face_info": (V, [P, ip, ip, ip]),
            "orc_cell_geom": (V, [P, dp, dp, dp, dp]),
            "orc_cell_ops": (V, [P, I, dp, dp, dp, dp, dp, ip]),
            "orc_face_mass": (V, [P, I, dp]),
            "orc_basis": (V, [P, I, D, D, dp, dp, dp]),
            "orc_face_basis": (V, [P, I, D, D, dp]),
            "orc_basis_many": (V, [P, I, ip, dp, dp, dp]),
            "orc_locate": (I, [P, D, D]),
            "orc_quad_count": (I, [P, I]),
            "orc_quad_points": (V, [P, I, dp, dp, dp, ip]),
            "orc_set_point_sources": (V, [P, I, dp, dp, dp, dp, dp]),
            "orc_set_dense_load": (V, [P, I, dp, dp, dp]),
            "orc_face_values": (V, [P, dp, dp]),
            "orc_rhs": (V, [P, dp, D, dp]),
            "orc_erk": (I, [P, I, dp, D, D, I, P]),
            "orc_energy": (D, [P, dp]),
            "orc_mass_dot": (D, [P, dp, dp]),
            "orc_stab_energy": (D, [P, dp]),
            "orc_point_values": (I, [P, dp, D, D, dp]),
            "orc_build_blocks": (V, [P]),
            "orc_keff": (V, [P, dp, dp]),
            "orc_keff_T": (V, [P, dp, dp, P]),
            "orc_inv_mass": (V, [P, dp, dp]),
            "orc_rhs_T": (V, [P, dp, dp]),
            "orc_grad_terms": (V, [P, dp, dp, dp, dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class Oracle:
    """FP64 reference discretisation of one mesh at polynomial degree k.

    eta_f, eta_s: stabilisation weights (0.8 and 1.5 in the paper, Sec. 5.1).
    stab_speed: the speed c^s in tau^s = rho c^s, which the paper leaves undefined: 1 (default)
    the S-wave speed, the reading under which the stability-optimal solid weight is the paper's
    eta^s = 1.5 (Sec. 5.1, Figure CFL_decoupled); 0 the P-wave speed.
    """

    def __init__(self, mesh, k, eta_f=0.8, eta_s=1.5, stab_speed=1):
        lib = _load()
        self.lib = lib
        self.mesh = mesh
        self.k = k
        self.N = (k + 1) * (k + 2) // 2
        self.nf = k + 1
        xy = np.ascontiguousarray(mesh["xy"], dtype=np.float64).reshape(-1)
        self.nc = len(mesh["cell_ptr"]) - 1
        self._h = lib.orc_create(len(xy) // 2, xy, self.nc,
                                 np.ascontiguousarray(mesh["cell_ptr"], np.int32),
                                 np.ascontiguousarray(mesh["cell_vtx"], np.int32),
                                 np.ascontiguousarray(mesh["medium"], np.uint8),
                                 np.ascontiguousarray(mesh["rho"], np.float64),
                                 np.ascontiguousarray(mesh["a"], np.float64),
                                 np.ascontiguousarray(mesh["b"], np.float64),
                                 int(k), float(eta_f), float(eta_s), int(stab_speed))
        if not self._h:
            raise ValueError("oracle: invalid mesh or parameters")
        self.ndof = lib.orc_ndof(self._h)
        self.offsets = np.zeros(self.nc + 1, np.int32)
        lib.orc_offsets(self._h, self.offsets)
        self.nfaces = lib.orc_nfaces(self._h)
        self.medium = np.asarray(mesh["medium"], np.uint8)

    def __del__(self):
        if getattr(self, "_h", None):
            self.lib.orc_destroy(self._h)
            self._h = None

    # ---------------------------------------------------------------- structure
    def face_info(self):
        fv = np.zeros(2 * self.nfaces, np.int32)
        fc = np.zeros(2 * self.nfaces, np.int32)
        tag = np.zeros(self.nfaces, np.int32)
        self.lib.orc_face_info(self._h, fv, fc, tag)
        return fv.reshape(-1, 2), fc.reshape(-1, 2), tag

    def face_offsets(self):
        off = np.zeros(self.nfaces + 1, np.int32)
        self.lib.orc_face_offsets(self._h, off)
        return off

    def cell_geom(self):
        a = np.zeros(self.nc)
        b = np.zeros(2 * self.nc)
        h = np.zeros(self.nc)
        t = np.zeros(self.nc)
        self.lib.orc_cell_geom(self._h, a, b, h, t)
        return dict(area=a, bary=b.reshape(-1, 2), h=h, eta_tau=t)

    def cell_ops(self, c):
        N, nf = self.N, self.nf
        m = int(self.mesh["cell_ptr"][c + 1] - self.mesh["cell_ptr"][c])
        M0 = np.zeros(N * N)
        D = np.zeros(2 * N * N)
        E = np.zeros(m * N * N)
        G = np.zeros(m * N * nf)
        n = np.zeros(2 * m)
        faces = np.zeros(m, np.int32)
        self.lib.orc_cell_ops(self._h, int(c), M0, D, E, G, n, faces)
        return dict(M0=M0.reshape(N, N), D=D.reshape(2, N, N), E=E.reshape(m, N, N),
                    G=G.reshape(m, N, nf), n=n.reshape(m, 2), faces=faces)

    def face_mass(self, f):
        MF = np.zeros(self.nf * self.nf)
        self.lib.orc_face_mass(self._h, int(f), MF)
        return MF.reshape(self.nf, self.nf)

    def basis(self, c, x, y):
        phi = np.zeros(self.N)
        px = np.zeros(self.N)
        py = np.zeros(self.N)
        self.lib.orc_basis(self._h, int(c), float(x), float(y), phi, px, py)
        return phi, px, py

    def basis_many(self, cells, x, y):
        cells = np.ascontiguousarray(cells, np.int32)
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        phi = np.zeros((len(cells), self.N))
        self.lib.orc_basis_many(self._h, len(cells), cells, x, y, phi)
        return phi

    def face_basis(self, f, x, y):
        psi = np.zeros(self.nf)
        self.lib.orc_face_basis(self._h, int(f), float(x), float(y), psi)
        return psi

    def locate(self, x, y):
        return self.lib.orc_locate(self._h, float(x), float(y))

    def quad_points(self, nq):
        n = self.lib.orc_quad_count(self._h, int(nq))
        px, py, pw = np.zeros(n), np.zeros(n), np.zeros(n)
        pc = np.zeros(n, np.int32)
        self.lib.orc_quad_points(self._h, int(nq), px, py, pw, pc)
        return px, py, pw, pc

    def ndof_cell(self):
        return np.diff(self.offsets)

    # ---------------------------------------------------------------- projections (L2(T))
    def project(self, fluid_fns, solid_fns, nq=None):
        """L2 projection of analytic fields onto the cell bases.

        fluid_fns: 3 callables (x, y) -> values for (p, m_x, m_y); solid_fns: 5
        callables for (v_x, v_y, s_1, s_2, s_3) in the E-basis components.
        """
        g = self.load_vector(fluid_fns, solid_fns, nq)
        return self.mass_solve_plain(g)

    def load_vector(self, fluid_fns, solid_fns, nq=None):
        """(f, phi_a)_T for every cell block (the load-vector reading of eq. rhs)."""
        nq = nq or self.k + 6
        px, py, pw, pc = self.quad_points(nq)
        N = self.N
        out = np.zeros(self.ndof)
        phi = self.basis_many(pc, px, py)
        med = self.medium[pc]
        for blk_fns, mcode, nb in ((fluid_fns, 0, 3), (solid_fns, 1, 5)):
            sel = med == mcode
            if not np.any(sel):
                continue
            for bl in range(nb):
                vals = blk_fns[bl](px[sel], py[sel]) * pw[sel]
                contrib = vals[:, None] * phi[sel]
                cells = pc[sel]
                idx = self.offsets[cells][:, None] + bl * N + np.arange(N)[None, :]
                np.add.at(out, idx.reshape(-1), contrib.reshape(-1))
        return out

    def mass_solve_plain(self, g):
        """Solve with the unweighted cell mass matrices M0 (block by block)."""
        out = np.zeros_like(g)
        N = self.N
        for c in range(self.nc):
            M0 = self.cell_ops(c)["M0"]
            nb = 3 if self.medium[c] == 0 else 5
            o = self.offsets[c]
            out[o:o + nb * N] = np.linalg.solve(M0, g[o:o + nb * N].reshape(nb, N).T).T.reshape(-1)
        return out

    # ---------------------------------------------------------------- loads
    def set_point_sources(self, xy, direction, f0, t0, amp):
        xy = np.ascontiguousarray(np.asarray(xy, np.float64).reshape(-1))
        n = len(xy) // 2
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(direction, np.float64), (n, 2)).reshape(-1))
        arr = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (n,)))
        self.lib.orc_set_point_sources(self._h, n, xy, d, arr(f0), arr(t0), arr(amp))

    def set_dense_load(self, g, omega, phase):
        g = np.ascontiguousarray(np.asarray(g, np.float64).reshape(-1))
        om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, np.float64)))
        ph = np.ascontiguousarray(np.atleast_1d(np.asarray(phase, np.float64)))
        self.lib.orc_set_dense_load(self._h, len(om), g if len(om) else np.zeros(1), om, ph)

    # ---------------------------------------------------------------- dynamics
    def rhs(self, U, t=0.0):
        U = np.ascontiguousarray(U, np.float64)
        out = np.zeros(self.ndof)
        self.lib.orc_rhs(self._h, U, float(t), out)
        return out

    def face_values(self, U):
        U = np.ascontiguousarray(U, np.float64)
        out = np.zeros(max(self.lib.orc_nface_dofs(self._h), 1))
        self.lib.orc_face_values(self._h, U, out)
        return out

    def erk(self, U, t0, dt, nsteps, s=4, energies=False):
        """Advance n steps of ERK(s) from t0; returns (U, E) with E[n] the energy after step n."""
        U = np.array(U, np.float64, copy=True)
        E = np.zeros(max(nsteps, 1)) if energies else None
        ptr = E.ctypes.data_as(C.c_void_p) if energies else None
        rc = self.lib.orc_erk(self._h, int(s), U, float(t0), float(dt), int(nsteps), ptr)
        if rc:
            raise ValueError("unsupported ERK stage count")
        return (U, E[:nsteps]) if energies else U

    def energy(self, U):
        return self.lib.orc_energy(self._h, np.ascontiguousarray(U, np.float64))

    def mass_dot(self, U, V):
        return self.lib.orc_mass_dot(self._h, np.ascontiguousarray(U, np.float64),
                                     np.ascontiguousarray(V, np.float64))

    def stab_energy(self, U):
        return self.lib.orc_stab_energy(self._h, np.ascontiguousarray(U, np.float64))

    def point_values(self, U, x, y):
        vals = np.zeros(5)
        c = self.lib.orc_point_values(self._h, np.ascontiguousarray(U, np.float64), float(x), float(y), vals)
        if c < 0:
            raise ValueError("point outside the mesh")
        nb = 3 if self.medium[c] == 0 else 5
        return c, vals[:nb]

    # ---------------------------------------------------------------- adjoint support
    def keff(self, z):
        """K_eff z from the explicit local blocks (K_T z + K_TF U_F, U_F = -K_F^{-1} K_FT z)."""
        out = np.zeros(self.ndof)
        self.lib.orc_keff(self._h, np.ascontiguousarray(z, np.float64), out)
        return out

    def keff_T(self, z):
        """K_eff^T z and the adjoint face values W_F = -K_F^{-T} K_TF^T z."""
        out = np.zeros(self.ndof)
        W = np.zeros(max(self.lib.orc_nface_dofs(self._h), 1))
        self.lib.orc_keff_T(self._h, np.ascontiguousarray(z, np.float64), out, W.ctypes.data_as(C.c_void_p))
        return out, W

    def inv_mass(self, x):
        out = np.zeros(self.ndof)
        self.lib.orc_inv_mass(self._h, np.ascontiguousarray(x, np.float64), out)
        return out

    def rhs_T(self, x):
        """L^T x for the condensed operator L = -M^{-1} K_eff."""
        out = np.zeros(self.ndof)
        self.lib.orc_rhs_T(self._h, np.ascontiguousarray(x, np.float64), out)
        return out

    def grad_terms(self, Y, k, mu, grad):
        """Accumulate mu^T (dL/dtheta) Y (+ the source part through k) into grad[n_cells, 3]."""
        assert grad.shape == (self.nc, 3) and grad.flags.c_contiguous
        self.lib.orc_grad_terms(self._h, np.ascontiguousarray(Y, np.float64), np.ascontiguousarray(k, np.float64),
                                np.ascontiguousarray(mu, np.float64), grad.reshape(-1))

    def dense_operator(self):
        """Columns of the condensed operator L = -M^{-1} K_eff (no loads), for tiny meshes."""
        Lmat = np.zeros((self.ndof, self.ndof))
        e = np.zeros(self.ndof)
        for j in range(self.ndof):
            e[:] = 0
            e[j] = 1.0
            Lmat[:, j] = self.rhs(e, 0.0)
        return Lmat
