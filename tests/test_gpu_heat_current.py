"""Heat current (Sec. II.E, eqs. Ji and J-1) of the HIP path vs the FP64 oracle.

J_i = W_i . v_i is linear in the per-atom virial, so its tolerance follows
from the virial's: |dJ_i,a| <= sum_b |dW_i,ab| |v_i,b| <= TOL_W * sum_b |v_i,b|
with TOL_W = 1e-4 eV the per-component bound of the float32 virial, and the
total within TOL_W * sum_i sum_b |v_i,b|.  The contraction itself runs in
float64 on the float32 virial, so it must also agree with W_i . v_i formed on
the host from the same library's per-atom virial to float64 rounding.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_10046_amd import nep, synth

pytestmark = pytest.mark.gpu

TOL_W = 1e-4  # eV, per-atom virial component of the float32 path


def log(*a):
    print(*a, flush=True)


def velocities(types, masses, seed):
    return synth.maxwell_velocities(np.asarray(masses)[types], 300.0, seed=seed)


def structures():
    rng = np.random.default_rng(91)
    return [
        ("fcc500_alloy4", synth.WORKLOADS["fcc131k"],
         synth.lattice("fcc", 5, 4.05, 0.1, 4, seed=11), synth.MASSES["fcc131k"]),
        ("triclinic130_train3", synth.WORKLOADS["train3"],
         synth.random_cell(130, 0.07, 0.2, 1.5, 3, rng), synth.MASSES["train3"]),
    ]


CASES = structures()


@pytest.fixture(scope="module")
def handles():
    cache = {}

    def get(name, h):
        if name not in cache:
            p = synth.random_params(O.num_params(h), seed=synth.SEED_WEIGHTS)
            cache[name] = (nep.Handle(h, p), p)
        return cache[name]
    return get


@pytest.mark.parametrize("name,h,struct,masses", CASES, ids=[c[0] for c in CASES])
def test_heat_current_matches_oracle(name, h, struct, masses, handles):
    pos, types, box = struct
    handle, p = handles(name, h)
    vel = velocities(types, masses, seed=7)
    n = pos.shape[1]
    log(f"[heat] {name} N={n}")
    J, T = handle.heat_current(pos, vel, types, box)
    Ja, J1, J2 = O.heat_current(h, p, pos, vel, types, box)
    bound = TOL_W * np.abs(vel).sum(axis=0)
    dJ = np.abs(J - Ja).max(axis=0)
    log(f"[heat] {name}: max|dJ_i|={dJ.max():.2e} (bound {bound.min():.2e}..{bound.max():.2e}) "
        f"|dJ|={np.abs(T - J1).max():.2e} |J1-J2|={np.abs(J1 - J2).max():.2e}")
    assert np.all(dJ <= bound)
    assert np.all(np.abs(T - J1) <= TOL_W * np.abs(vel).sum())
    # the total is the float64 sum of the per-atom currents
    np.testing.assert_allclose(T, J.sum(axis=1), rtol=0, atol=1e-12 * np.abs(J).sum())
    # and each J_i is W_i . v_i of the library's own per-atom virial
    W = handle.compute(pos, types, box)["W"].reshape(3, 3, n)
    np.testing.assert_allclose(J, np.einsum("abn,bn->an", W, vel), rtol=0,
                               atol=1e-13 * np.abs(W).max() * np.abs(vel).max())


def test_heat_current_zero_velocity_and_repeatable(handles):
    name, h, (pos, types, box), masses = CASES[0]
    handle, _ = handles(name, h)
    J0, T0 = handle.heat_current(pos, np.zeros_like(pos), types, box)
    assert not np.any(J0) and not np.any(T0)
    vel = velocities(types, masses, seed=8)
    a = handle.heat_current(pos, vel, types, box)
    b = handle.heat_current(pos, vel, types, box)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_heat_current_device_entry_matches_host(handles):
    import torch
    name, h, (pos, types, box), masses = CASES[1]
    handle, _ = handles(name, h)
    vel = velocities(types, masses, seed=9)
    J, T = handle.heat_current(pos, vel, types, box)
    dev = torch.device("cuda:0")
    n = pos.shape[1]
    heat = torch.zeros(3, n, dtype=torch.float64, device=dev)
    tot = torch.zeros(3, dtype=torch.float64, device=dev)
    handle.heat_current_dev(torch.tensor(pos, device=dev), torch.tensor(vel, device=dev),
                            torch.tensor(types, device=dev), box, heat=heat, total=tot)
    torch.cuda.synchronize()
    assert np.array_equal(heat.cpu().numpy(), J)
    assert np.array_equal(tot.cpu().numpy(), T)


def test_heat_current_errors(handles):
    name, h, (pos, types, box), masses = CASES[0]
    handle, _ = handles(name, h)
    vel = velocities(types, masses, seed=10)
    bad = vel.copy()
    bad[1, 3] = np.nan
    with pytest.raises(nep.NepError):
        handle.heat_current(pos, bad, types, box)


def test_heat_current_full_size_fcc131k_sampled(handles):
    """The 131,072-atom alloy at 300 K: sampled atoms vs the oracle's W_i . v_i."""
    h = synth.WORKLOADS["fcc131k"]
    pos, types, box = synth.fcc131k()
    handle, p = handles("fcc131k", h)
    vel = velocities(types, synth.MASSES["fcc131k"], seed=11)
    log(f"[heat] fcc131k N={pos.shape[1]}")
    J, T = handle.heat_current(pos, vel, types, box)
    idx = np.random.default_rng(12).choice(pos.shape[1], 12, replace=False)
    W = O.evaluate_atoms(h, p, pos, types, box, idx)["W"].reshape(-1, 3, 3)
    ref = np.einsum("kab,kb->ka", W, vel[:, idx].T)
    dJ = np.abs(J[:, idx].T - ref).max(axis=1)
    bound = TOL_W * np.abs(vel[:, idx]).sum(axis=0)
    log(f"[heat] fcc131k sampled: max|dJ_i|={dJ.max():.2e}")
    assert np.all(dJ <= bound)
    np.testing.assert_allclose(T, J.sum(axis=1), rtol=0, atol=1e-12 * np.abs(J).sum())
