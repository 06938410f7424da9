"""SNES steps on the GPU (the trainer of Sec. II.E) vs the FP64 oracle.

Both sides rank the same float64 losses with the same tie rule, so the ranks
agree exactly; the utilities use log and the scale step exp, whose float64
results may differ by an ulp between the device and the host library, and the
sums over members may be fused differently: every result is compared to a
relative 1e-12.  The sampled population is one multiply-add per entry.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_10046_amd import nep, synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def handle():
    h = synth.WORKLOADS["train3"]
    p = synth.random_params(O.num_params(h))
    return h, p, nep.Handle(h, p)


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.mark.parametrize("P,stride", [(50, 1), (7, 6), (2, 1), (1024, 1)])
def test_snes_step_matches_oracle(handle, P, stride):
    import torch
    h, _, hd = handle
    d = O.num_params(h)
    rng = np.random.default_rng(100 + P)
    mean, sigma = rng.normal(0, 0.1, d), rng.uniform(0.05, 0.2, d)
    noise = rng.normal(size=(P, d))
    losses = rng.uniform(0.1, 1.0, P)
    losses[P // 2] = losses[0]  # a tie, broken by index on both sides
    buf = np.full((P, stride), np.nan)
    buf[:, 0] = losses
    eta = O.snes_rates(d)
    tm, ts = _t(mean), _t(sigma)
    log(f"[snes] P={P} d={d} stride={stride}")
    hd.snes_step(tm, ts, _t(noise), _t(buf), *eta, loss_stride=stride)
    torch.cuda.synchronize()
    rm, rs = O.snes_step(mean, sigma, noise, losses, *eta)
    np.testing.assert_allclose(tm.cpu().numpy(), rm, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(ts.cpu().numpy(), rs, rtol=1e-12)


def test_snes_step_ranks_non_finite_losses_last(handle):
    """A diverged member (NaN or Inf loss) ranks after every finite one on
    the device as in the oracle, so the update stays that of a permutation
    of utilities."""
    import torch
    h, _, hd = handle
    d, P = O.num_params(h), 9
    rng = np.random.default_rng(150)
    mean, sigma = rng.normal(0, 0.1, d), rng.uniform(0.05, 0.2, d)
    noise = rng.normal(size=(P, d))
    losses = rng.uniform(0.1, 1.0, P)
    losses[2], losses[5], losses[7] = np.nan, np.inf, np.nan
    eta = O.snes_rates(d)
    tm, ts = _t(mean), _t(sigma)
    hd.snes_step(tm, ts, _t(noise), _t(losses), *eta)
    torch.cuda.synchronize()
    rm, rs = O.snes_step(mean, sigma, noise, losses, *eta)
    assert np.isfinite(tm.cpu().numpy()).all()
    np.testing.assert_allclose(tm.cpu().numpy(), rm, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(ts.cpu().numpy(), rs, rtol=1e-12)


def test_snes_sample_matches_oracle(handle):
    import torch
    h, _, hd = handle
    d, P = O.num_params(h), 13
    rng = np.random.default_rng(120)
    mean, sigma, noise = rng.normal(size=d), rng.uniform(0.1, 1.0, d), rng.normal(size=(P, d))
    pop = torch.zeros(P, d, dtype=torch.float64, device="cuda:0")
    hd.snes_sample(_t(mean), _t(sigma), _t(noise), pop)
    torch.cuda.synchronize()
    ref = O.snes_sample(mean, sigma, noise)
    np.testing.assert_allclose(pop.cpu().numpy(), ref, rtol=0, atol=4e-16 * np.abs(ref).max())


def test_snes_generations_on_device(handle):
    """Three generations of sample -> batch evaluation -> loss -> step, all
    on the device; each step equals the oracle's step applied to the losses
    the device computed, and the losses equal the loss of each member."""
    import torch
    h, p0, hd = handle
    d, P = O.num_params(h), 6
    structs = synth.random_structures(5, 8, 40, seed=130)
    pos, types, boxes, offs = synth.concat_structures(structs)
    teacher = synth.random_params(d, seed=131)
    e_t, f_t, w_t = O.predictions(h, teacher, structs)
    n, S = pos.shape[1], boxes.shape[0]
    dev = torch.device("cuda:0")
    tp, tt = torch.tensor(pos, device=dev), torch.tensor(types, device=dev)
    te, tf, tw = _t(e_t), _t(f_t), _t(w_t)
    mean, sigma = _t(p0), _t(np.full(d, 0.05))
    eta = O.snes_rates(d)
    lam = (1.0, 1.0, 0.1, 1e-4, 1e-4)
    rng = np.random.default_rng(132)
    for g in range(3):
        noise = rng.normal(size=(P, d))
        tn = _t(noise)
        pop = torch.zeros(P, d, dtype=torch.float64, device=dev)
        hd.snes_sample(mean, sigma, tn, pop)
        f = torch.zeros(P, 3, n, dtype=torch.float64, device=dev)
        t = torch.zeros(P, S, 10, dtype=torch.float64, device=dev)
        zh = pop.cpu().numpy()
        hd.compute_batch(offs, tp, tt, boxes, zh, None, f, None, t)
        loss = torch.zeros(P, 6, dtype=torch.float64, device=dev)
        hd.batch_loss(offs, f, t, te, tf, lam, loss, virial_target=tw, params=pop)
        m0, s0 = mean.cpu().numpy(), sigma.cpu().numpy()
        hd.snes_step(mean, sigma, tn, loss, *eta, loss_stride=6)
        torch.cuda.synchronize()
        L = loss.cpu().numpy()[:, 0]
        rm, rs = O.snes_step(m0, s0, noise, L, *eta)
        log(f"[snes] generation {g}: losses {np.round(L, 4)}")
        np.testing.assert_allclose(mean.cpu().numpy(), rm, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(sigma.cpu().numpy(), rs, rtol=1e-12)
        np.testing.assert_allclose(zh, O.snes_sample(m0, s0, noise), rtol=0,
                                   atol=4e-16 * np.abs(zh).max())


def test_snes_rejects_bad_sizes(handle):
    _, _, hd = handle
    import torch
    z = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(nep.NepError):
        hd.snes_step(z, z, z.reshape(1, 4), z, 1.0, 0.1)  # one member: no ranking
