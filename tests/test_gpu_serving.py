"""The continuous-batching server: results against the oracle, and each
request's result alone equal (bitwise) to its result in a mix of requests
that arrive while others are on the GPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_10046_amd import nep, synth

pytestmark = pytest.mark.gpu

H = synth.WORKLOADS["serve2"]
MASSES = np.array(synth.MASSES["serve2"])


def log(*a):
    print(*a, flush=True)


def requests(seed=9):
    rng = np.random.default_rng(seed)
    out = []
    for k, (kind, a, nc) in enumerate([("fcc", 4.05, 3), ("bcc", 3.16, 4), ("fcc", 4.05, 4),
                                        ("bcc", 3.16, 3), ("fcc", 4.05, 5), ("bcc", 3.16, 5)]):
        pos, types, box = synth.lattice(kind, nc, a, 0.05, 2, seed=int(rng.integers(1 << 30)))
        if k % 2:
            vel = synth.maxwell_velocities(MASSES[types], 300.0, seed=int(rng.integers(1 << 30)))
            out.append(dict(pos=pos, types=types, box=box, kind=nep.NEP_REQ_MD, vel=vel,
                            masses=MASSES, n_steps=5 + k))
        else:
            out.append(dict(pos=pos, types=types, box=box, kind=nep.NEP_REQ_EVAL))
    return out


@pytest.fixture(scope="module")
def server():
    params = synth.random_params(O.num_params(H))
    srv = nep.Server(nep.Handle(H, params), 8 << 30, max_slots=16)
    yield srv, params
    srv.close()


def test_server_results_match_oracle(server):
    srv, params = server
    reqs = requests()
    tickets = [srv.submit(**r) for r in reqs]
    for r, t in zip(reqs, tickets):
        res = srv.poll(t, wait_ms=-1)
        if r["kind"] == nep.NEP_REQ_EVAL:
            ref = O.evaluate(H, params, r["pos"], r["types"], r["box"])
            dU = np.abs(res["U"] - ref["U"]).max()
            dF = np.abs(res["F"] - ref["F"]).max()
            log(f"[serve] eval N={r['pos'].shape[1]} |dU|={dU:.2e} |dF|={dF:.2e} "
                f"latency {res['latency_ms']:.2f} ms")
            dE = abs(res["U"].sum() - ref["U"].sum()) / r["pos"].shape[1]
            assert dE <= 1e-6 and dU <= 1e-5 and dF <= 1e-4
        else:
            op, ov, _ = O.md_nve(H, params, r["pos"], r["vel"], r["types"], MASSES, r["box"],
                                 1.0, r["n_steps"], 0)
            dp = np.abs(res["pos"] - op).max()
            log(f"[serve] md N={r['pos'].shape[1]} steps={r['n_steps']} |dr|={dp:.2e}")
            assert dp < 1e-6
    st = srv.stats()
    log(f"[serve] stats {st}")
    assert st["completed"] >= len(reqs)


def test_server_batch_invariance_bitwise(server):
    srv, _ = server
    reqs = requests(seed=4)
    alone = []
    for r in reqs:                       # one at a time: each runs alone in the batch
        alone.append(srv.poll(srv.submit(**r), wait_ms=-1))
    tickets = [srv.submit(**r) for r in reqs]   # all at once: they share ticks
    mixed = [srv.poll(t, wait_ms=-1) for t in tickets]
    assert srv.stats()["mean_batch_requests"] > 1.0
    for r, a, m in zip(reqs, alone, mixed):
        for k in ("U", "F", "W") + (("pos", "vel") if r["kind"] == nep.NEP_REQ_MD else ()):
            assert np.array_equal(a[k], m[k]), k


def test_server_rejects_over_budget():
    params = synth.random_params(O.num_params(H))
    srv = nep.Server(nep.Handle(H, params), 1 << 20, max_slots=4)
    pos, types, box = synth.lattice("fcc", 6, 4.05, 0.05, 2)
    with pytest.raises(nep.NepError) as e:
        srv.submit(pos, types, box)
    assert e.value.code == nep.NEP_E_BUDGET
    srv.close()
