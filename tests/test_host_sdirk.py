"""Host-side checks of the SDIRK plan (no GPU): the condensed face matrix that hho_sdirk_setup
builds equals the oracle's dense Schur complement a* dt (K_F - a* dt K_FT (M + a* dt K_T)^{-1} K_TF)
of its globally assembled operator (Sec. 4.1, the solves following eq. cp_dirk), face unknowns
matched by their face's vertices and their index in the face block; and bad input is refused."""
import numpy as np
import pytest

import synth.meshes as M
from oracle.implicit import ImplicitOracle, sdirk_tableau
from paper_2505_15771_amd import hho


def _mesh():
    ref = np.zeros((3, 3), bool)
    ref[0, 1] = True
    return M.with_materials(M.unit_square(3, p_split=0.5, seed=11, refine=ref), perturb=0.1, seed=12)


def _dense(ptr, col, val):
    n = len(ptr) - 1
    S = np.zeros((n, n))
    for d in range(n):
        S[d, col[ptr[d]:ptr[d + 1]]] = val[ptr[d]:ptr[d + 1]]
    return S


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("mixed", [True, False])
@pytest.mark.parametrize("stages,alpha,stab_speed", [(3, 1, 0), (1, 0, 1), (2, 1, 1)])
def test_face_matrix_matches_oracle_schur_complement(k, mixed, stages, alpha, stab_speed):
    m = _mesh()
    dt = 0.05
    io = ImplicitOracle(m, k, mixed=mixed, alpha=alpha, eta_f=0.9, eta_s=1.3, stab_speed=stab_speed)
    A, _, _ = sdirk_tableau(stages)
    adt = A[0, 0] * dt
    K = io.K.toarray()
    nd = io.ndof
    KT, KTF, KFT, KF = K[:nd, :nd], K[:nd, nd:], K[nd:, :nd], K[nd:, nd:]
    S_ref = adt * (KF - adt * KFT @ np.linalg.solve(io.M.toarray() + adt * KT, KTF))
    ptr, col, val, face = hho.sdirk_face_matrix(m, k, dt, stages=stages, mixed=mixed, alpha=alpha, eta_f=0.9,
                                                eta_s=1.3, stab_speed=stab_speed)
    key = {}
    for f in range(len(io.ftag)):
        for i in range(int(io.foff[f + 1] - io.foff[f])):
            key[(int(io.fv[f, 0]), int(io.fv[f, 1]), i)] = int(io.foff[f]) - nd + i
    perm = np.array([key[tuple(int(v) for v in face[d])] for d in range(len(face))])
    assert len(perm) == io.nface_dofs and len(set(perm)) == len(perm)
    S = _dense(ptr, col, val)
    S_ref = S_ref[np.ix_(perm, perm)]
    assert np.abs(S - S_ref).max() <= 1e-13 * np.abs(S_ref).max()


@pytest.mark.parametrize("k", [1, 3])
def test_face_matrix_with_physical_materials(k):
    """Granite (rho 2690, cP 6000 m/s) under water (rho 1025, c 1500 m/s) on a coarse bilayer: mass
    entries from 1/kappa ~ 4e-10 to rho ~ 3e3 in one stage matrix.  The plan's per-cell inverses
    are scaled so that this spread is harmless; the face matrix still equals the oracle's."""
    m = M.granite_water(nx=6, ny_s=3, ny_f=2)
    dt = 0.398 * 3800.0 / 6 / 6000.0
    io = ImplicitOracle(m, k)
    A, _, _ = sdirk_tableau(3)
    adt = A[0, 0] * dt
    K = io.K.toarray()
    nd = io.ndof
    KT, KTF, KFT, KF = K[:nd, :nd], K[:nd, nd:], K[nd:, :nd], K[nd:, nd:]
    S_ref = adt * (KF - adt * KFT @ np.linalg.solve(io.M.toarray() + adt * KT, KTF))
    ptr, col, val, face = hho.sdirk_face_matrix(m, k, dt)
    key = {}
    for f in range(len(io.ftag)):
        for i in range(int(io.foff[f + 1] - io.foff[f])):
            key[(int(io.fv[f, 0]), int(io.fv[f, 1]), i)] = int(io.foff[f]) - nd + i
    perm = np.array([key[tuple(int(v) for v in face[d])] for d in range(len(face))])
    S = _dense(ptr, col, val)
    S_ref = S_ref[np.ix_(perm, perm)]
    # row-wise relative comparison: fluid and solid rows differ by orders of magnitude
    scale = np.abs(S_ref).max(axis=1, keepdims=True)
    assert (np.abs(S - S_ref) <= 1e-12 * scale).all()


def test_given_domain_length_scales_the_weights():
    """alpha = 1 with l_Omega given explicitly equal to the diameter gives the same matrix as the
    computed diameter (sqrt 2 for the unit square); another l_Omega changes it."""
    m = _mesh()
    a = hho.sdirk_face_matrix(m, 1, 0.05)[2]
    b = hho.sdirk_face_matrix(m, 1, 0.05, ell=np.sqrt(2.0))[2]
    c = hho.sdirk_face_matrix(m, 1, 0.05, ell=3.0)[2]
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    assert np.abs(a - c).max() > 1e-3 * np.abs(a).max()


@pytest.mark.parametrize("kw,code", [(dict(stages=4), 1), (dict(stages=0), 1), (dict(k=4), 1), (dict(k=0), 1),
                                     (dict(dt=0.0), 1), (dict(dt=float("nan")), 1), (dict(alpha=2), 1),
                                     (dict(mixed=2), 1), (dict(ell=-1.0), 1), (dict(eta_f=0.0), 1),
                                     (dict(stab_speed=2), 1)])
def test_rejects_bad_parameters(kw, code):
    args = dict(k=1, dt=0.05)
    args.update(kw)
    with pytest.raises(hho.HHOError) as e:
        hho.sdirk_face_matrix(_mesh(), **args)
    assert e.value.code == code


def test_rejects_bad_mesh():
    m = _mesh()
    bad = dict(m)
    bad["cell_vtx"] = m["cell_vtx"][::-1].copy()   # clockwise / mismatched
    with pytest.raises(hho.HHOError) as e:
        hho.sdirk_face_matrix(bad, 1, 0.05)
    assert e.value.code == 2
