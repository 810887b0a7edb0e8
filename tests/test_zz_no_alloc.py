"""GPU check of hho_energy_noalloc (the energy entry point for callers that cannot allocate device
memory) through the C ABI: on two calls in a row, the second on a smaller context, its energies
equal those of hho_energy (same kernels, same summation order); a context whose partial sums
exceed the static scratch is refused on the host before any launch."""
import ctypes as C
import sys

import numpy as np
import pytest

from synth import meshes as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(mesh, k, shots, dtype, seed):
    from paper_2505_15771_amd import Engine
    e = Engine(mesh, k, dtype=dtype, n_shots=shots)
    rng = np.random.default_rng(seed)
    for sh in range(shots):
        e.set_state(rng.standard_normal(e.n_dof), shot=sh)
    return e


def _noalloc(e):
    import torch
    out = torch.full((e.n_shots,), float("nan"), dtype=torch.float64, device="cuda")
    code = e.lib.hho_energy_noalloc(e._h, C.c_void_p(out.data_ptr()))
    assert code == 0, e.lib.hho_last_error(e._h).decode()
    e.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_energy_noalloc_matches_energy(dtype):
    say("case: hho_energy_noalloc, larger then smaller context,", dtype)
    big = _engine(M.hanging_square(24, seed=4), 2, 3, dtype, 11)
    small = _engine(M.with_materials(M.unit_square(6, p_split=0.5, seed=2)), 1, 1, dtype, 12)
    for e in (big, small):
        ref = e.energy()
        got = _noalloc(e)
        say("  shots", e.n_shots, "hho_energy", ref, "noalloc", got)
        assert np.all(np.isfinite(got)) and np.all(ref > 0)
        assert np.max(np.abs(got - ref) / ref) <= 1e-15
    # after stepping the larger context, the shared scratch still gives its energies
    big.erk_step(0.0, big.dt_cfl(0.5), 3)
    assert np.max(np.abs(_noalloc(big) - big.energy()) / big.energy()) <= 1e-15
    big.close()
    small.close()


def test_energy_noalloc_refuses_oversized_context():
    """256 shots of a 40 x 40 quad mesh: 1600 cells x 256 partial sums > 262144; refused with ARG
    on the host (no kernel runs), and the context still works."""
    say("case: hho_energy_noalloc size limit")
    e = _engine(M.with_materials(M.unit_square(40)), 1, 256, "f32", 13)
    import torch
    out = torch.zeros(256, dtype=torch.float64, device="cuda")
    code = e.lib.hho_energy_noalloc(e._h, C.c_void_p(out.data_ptr()))
    assert code == 1 and "scratch" in e.lib.hho_last_error(e._h).decode()
    assert np.all(e.energy() > 0)
    e.close()
