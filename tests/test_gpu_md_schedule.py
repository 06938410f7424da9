"""Row maintenance of MD with a skin (nep_md_run*): a captured group of steps
checks for a rebuild at its first step only, looking ahead by 1.5 times each
atom's speed over the group; every later step verifies the skin, and a chunk
in which an atom left it is replayed step by step from its saved state.
Either way the trajectory is that of rows rebuilt from scratch every step,
to float32 summation order."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_10046_amd import nep, synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def hot_cell():
    h = synth.WORKLOADS["fcc131k"]
    p = synth.random_params(O.num_params(h))
    pos, types, box = synth.lattice("fcc", 8, 4.05, 0.05, 4, seed=21)
    m = np.array(synth.MASSES["fcc131k"])
    vel = synth.maxwell_velocities(m[types], 900.0, seed=22)
    return h, p, pos, vel, types, m, box


def _run(h, p, skin, args, lookahead=None):
    old = os.environ.get("NEP_MD_LOOKAHEAD")
    if lookahead is not None:
        os.environ["NEP_MD_LOOKAHEAD"] = str(lookahead)
    try:
        handle = nep.Handle(h, p, skin=skin)
        out = handle.md_run(*args)
        cnt = handle.md_counters()
        handle.close()
    finally:
        if lookahead is not None:
            if old is None:
                del os.environ["NEP_MD_LOOKAHEAD"]
            else:
                os.environ["NEP_MD_LOOKAHEAD"] = old
    return out, cnt


@pytest.mark.parametrize("skin,lookahead", [(0.5, None), (0.1, 0.0)],
                         ids=["skin0.5-default", "skin0.1-no-lookahead"])
def test_grouped_rebuild_checks_match_rows_from_scratch(hot_cell, skin, lookahead):
    h, p, pos, vel, types, m, box = hot_cell
    args = (pos, vel, types, m, box, 1.0, 200, 10)
    (pa, va, tha), _ = _run(h, p, 0.0, args)
    (pb, vb, thb), cnt = _run(h, p, skin, args, lookahead)
    dp = np.abs(pa - pb).max()
    log(f"[schedule] skin {skin}, look-ahead {lookahead}: {cnt}, max|dr| vs rows from scratch {dp:.2e}")
    if lookahead == 0.0:
        # a 0.05 A allowance at 900 K is crossed inside groups: chunks are replayed
        assert cnt["replayed_chunks"] > 0
    else:
        assert cnt["group_steps"] > 0
    assert dp < 1e-6
    np.testing.assert_allclose(tha[:, 1:3], thb[:, 1:3], atol=1e-6 * pos.shape[1])


def test_continued_runs_reuse_the_state_and_match_one_run(hot_cell):
    """Ten calls of 20 steps, each fed the previous call's output, keep the
    atom order, rows and forces of the call before (no set-up in between) and
    give the trajectory of one 200-step call bit for bit; a call whose
    positions differ from the returned ones, or that follows another call on
    the handle, sets up anew."""
    h, p, pos, vel, types, m, box = hot_cell
    one = nep.Handle(h, p, skin=0.5)
    p1, v1, th1 = one.md_run(pos, vel, types, m, box, 1.0, 200, 10)
    one.close()
    split = nep.Handle(h, p, skin=0.5)
    pc, vc, rows = pos, vel, []
    for _ in range(10):
        pc, vc, th = split.md_run(pc, vc, types, m, box, 1.0, 20, 10)
        rows.append(th)
    cnt = split.md_counters()
    log(f"[continue] split into 10 calls: {cnt}")
    assert cnt["continued_runs"] == 9
    assert np.array_equal(pc, p1) and np.array_equal(vc, v1)
    assert np.array_equal(np.concatenate(rows)[:, 1:], th1[:, 1:])
    # a moved atom: set up again, and the result is a fresh handle's
    moved = pc.copy()
    moved[0, 5] += 1e-3
    pm, vm, _ = split.md_run(moved, vc, types, m, box, 1.0, 20, 10)
    assert split.md_counters()["continued_runs"] == 9
    fresh = nep.Handle(h, p, skin=0.5)
    pf, vf, _ = fresh.md_run(moved, vc, types, m, box, 1.0, 20, 10)
    fresh.close()
    assert np.abs(pm - pf).max() < 1e-6
    # another call in between: set up again
    split.compute(pm, types, box)
    split.md_run(pm, vm, types, m, box, 1.0, 20, 10)
    assert split.md_counters()["continued_runs"] == 9
    split.close()
