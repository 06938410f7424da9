"""Host replay of the evaluation kernels' address arithmetic (no GPU).

For the 40-atom triclinic 3-species structure of the training-batch model
(several periodic images per pair, so image codes are read), this replays on
the CPU, thread by thread, the index expressions of the descriptor, network,
partial-force and gather kernels for every (angular group size, block size,
lanes per atom) shape the autotuner launches, on rows in the library's layout
(the angular entries first, then the outer ones) built from the oracle's pair
search, and checks that every global and LDS access lies inside the buffer the
library allocates for it.  The GPU checks the row invariants this relies on
(k_check_rows) before any evaluation kernel runs.

The replay mirrors the kernels' loops: the software-pipelined neighbour loads
(entries up to two steps ahead; past the row they read atom 0), the clamped
prefetches of the gather, the per-lane LDS slots, and the network tile loads.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2205_10046_amd import synth

XCDS = 8


def xcd_block(b, nb):
    x, k, q, r = b % XCDS, b // XCDS, nb // XCDS, nb % XCDS
    return x * q + min(x, r) + k


def ng_pad(ng):
    return ng if ng <= 2 else (ng + 3) // 4 * 4


def round4(n):
    return (n + 3) // 4 * 4


def pair_stride(n):
    return n + ((4 - n % 64) + 64) % 64


def group_options(nA, L):
    cap = 7 if L <= 4 else (5 if L == 5 else 4)
    out = [ng for ng in (2, 4, 5, 7) if ng <= cap and (ng <= nA or ng == 2)]
    return out or [2]


def estimate_capacity(rc, density):
    m = math.ceil(1.3 * 4.0 / 3.0 * math.pi * rc ** 3 * density + 24)
    return (m + 3) // 4 * 4


class Bounds:
    def __init__(self, sizes):
        self.sizes = sizes
        self.hi = {k: -1 for k in sizes}
        self.lo = {k: 0 for k in sizes}

    def touch(self, buf, idx):
        idx = int(idx)
        self.hi[buf] = max(self.hi[buf], idx)
        self.lo[buf] = min(self.lo[buf], idx)

    def check(self, what):
        for k, n in self.sizes.items():
            assert self.lo[k] >= 0, (what, k, self.lo[k])
            assert self.hi[k] < n, (what, k, self.hi[k], n)


def library_rows(pos, box, rcR, rcA):
    """Exact rows in the library's layout: angular-range entries first, then
    the outer ones, each part in (j, image) order; rev[i][m] = position of i
    in the row of its m-th neighbour."""
    R = O.pairs(pos, box, rcR)
    H = box.reshape(3, 3)
    rows = []
    for i, (j, sh) in enumerate(R):
        d = (pos[:, j] - pos[:, [i]]).T + sh @ H
        r2 = (d ** 2).sum(1)
        inner = [k for k in range(len(j)) if r2[k] < rcA * rcA]
        outer = [k for k in range(len(j)) if r2[k] >= rcA * rcA]
        order = inner + outer
        rows.append((j[order], sh[order], len(inner)))
    rev = []
    for i, (j, sh, _) in enumerate(rows):
        rv = []
        for jj, s in zip(j, sh):
            jr, sr, _ = rows[jj]
            hit = [k for k in range(len(jr)) if jr[k] == i and np.array_equal(sr[k], -s)]
            assert len(hit) == 1
            rv.append(hit[0])
        rev.append(rv)
    return rows, rev


def for_entries(b, N, i, first, nn, step, nl_row):
    """The entries a lane visits and the global reads of its pipelined loop."""
    def index_of(m):
        if m >= nn:
            return 0
        b.touch("nl", m * N + i)
        b.touch("cd", m * N + i)
        return nl_row[m]
    j0 = index_of(first)
    index_of(first + step)
    for c in range(3):
        b.touch("pos", c * N + j0)
    b.touch("types", j0)
    out = []
    m = first
    while m < nn:
        out.append(m)
        nxt = index_of(m + step) if m + step < nn else 0
        for c in range(3):
            b.touch("pos", c * N + nxt)
        b.touch("types", nxt)
        index_of(m + 2 * step)
        m += step
    return out


def replay_pair(N, capN, rows, rev, types, M, NG, block, G, force):
    T, nR, KR, nA, KA, L, NB, NDp = (M[k] for k in ("T", "nR", "KR", "nA", "KA", "L", "NB", "NDp"))
    MR = M["MR"]
    W = ng_pad(NG)
    groups = -(-nA // NG)
    cA_pair = pair_stride(groups * KA * W)
    lds_floats = (round4(T * T * nR * KR) + round4(M["cA_max"]) + T * KR * block)
    sR0, sA0 = 0, round4(T * T * nR * KR)
    acc0 = sA0 + round4(T * T * cA_pair)
    b = Bounds(dict(nl=MR * capN, cd=MR * capN, rev=MR * capN, P=MR * capN, pos=3 * capN,
                    types=capN, sums=nA * NB * capN, q=capN * NDp, fp=capN * NDp,
                    lds=lds_floats, sR=T * T * nR * KR, sA=T * T * cA_pair))
    nb = -(-N * G // block)
    for blk in range(nb):
        xb = xcd_block(blk, nb)
        for tid in range(block):
            i = (xb * block + tid) // G
            if i >= N:
                continue
            sub = tid % G
            j, _, nnA = rows[i]
            nnR = len(j)
            ti = types[i]
            for t in range(T):
                for k in range(KR):
                    b.touch("lds", acc0 + (t * KR + k) * block + tid)
            if not force:
                for m in for_entries(b, N, i, sub, nnR, G, j):
                    b.touch("lds", acc0 + (types[j[m]] * KR + KR - 1) * block + tid)
                for t in range(T):
                    for k in range(KR):
                        for n in range(nR):
                            b.touch("sR", (ti * T + t) * nR * KR + k + n * KR)
                for n in range(nR):
                    b.touch("q", i * NDp + n)
                for g in range(groups):
                    for m in for_entries(b, N, i, sub, nnA, G, j):
                        base = (ti * T + types[j[m]]) * cA_pair + g * KA * W
                        for k in range(KA):
                            b.touch("sA", base + k * W)
                            b.touch("sA", base + k * W + W - 1)
                    for q in range(NG):
                        n = g * NG + q
                        if n >= nA:
                            break
                        for k in range(NB):
                            b.touch("sums", (n * NB + k) * N + i)
                b.touch("q", i * NDp + NDp - 1)
            else:
                for n in range(nR):
                    b.touch("fp", i * NDp + n)
                m_outer = sub + ((nnA - sub + G - 1) // G * G if nnA > sub else 0)
                for m in for_entries(b, N, i, m_outer, nnR, G, j):
                    b.touch("P", m * N + i)
                for g in range(groups):
                    for q in range(NG):
                        n = min(g * NG + q, nA - 1)
                        for k in range(NB):
                            b.touch("sums", (n * NB + k) * N + i)
                        if g * NG + q < nA:
                            b.touch("fp", i * NDp + nR + (L - 1) * nA + n)
                            b.touch("fp", i * NDp + nR + (L + M["has4b"] + M["has5b"] - 1) * nA + n)
                    for m in for_entries(b, N, i, sub, nnA, G, j):
                        base = (ti * T + types[j[m]]) * cA_pair + g * KA * W
                        b.touch("sA", base + (KA - 1) * W + W - 1)
                        b.touch("P", m * N + i)
    # the gather: dU_j/dr_ji at rev[m][i] of row j, prefetched one entry ahead
    if force:
        nbg = -(-N * G // 256)
        for blk in range(nbg):
            xb = xcd_block(blk, nbg)
            for tid in range(256):
                i = (xb * 256 + tid) // G
                if i >= N:
                    continue
                sub = tid % G
                j, _, _ = rows[i]
                nn = len(j)
                for m in list(range(sub, nn, G)) + [sub, sub + G]:
                    mm = min(m, max(nn - 1, 0))
                    b.touch("P", mm * N + i)
                    if m < nn:
                        b.touch("rev", m * N + i)
                        b.touch("P", rev[i][m] * N + j[m])
                        for c in range(3):
                            b.touch("pos", c * N + j[m])
    assert b.sizes["lds"] * 4 <= 64 * 1024
    b.check((NG, block, G, "force" if force else "descriptor"))
    return b


def test_train3_triclinic40_every_autotuned_shape_in_bounds():
    h = synth.WORKLOADS["train3"]
    rng = np.random.default_rng(77)
    # the same structure as the GPU parity case triclinic40_train3
    synth.random_cell(8, 0.07, 0.2, 1.5, 3, rng)
    pos, types, box = synth.random_cell(40, 0.07, 0.2, 1.5, 3, rng)
    N = pos.shape[1]
    rows, rev = library_rows(pos, box, h["rc_radial"], h["rc_angular"])
    vol = abs(np.linalg.det(box.reshape(3, 3)))
    MR = estimate_capacity(h["rc_radial"], N / vol)
    assert max(len(r[0]) for r in rows) <= MR
    assert all(len(set(r[0].tolist())) < len(r[0]) for r in rows)  # several images per pair
    T, L = h["n_types"], h["l_max_3b"]
    nA, KA = h["n_max_angular"] + 1, h["basis_angular"] + 1
    nd = O.num_descriptors(h)
    M = dict(T=T, nR=h["n_max_radial"] + 1, KR=h["basis_radial"] + 1, nA=nA, KA=KA, L=L,
             NB=(L + 1) ** 2 - 1, NDp=(nd + 7) // 8 * 8, MR=MR, has4b=int(h["l_max_4b"] >= 2),
             has5b=int(h["l_max_5b"] >= 1))
    M["cA_max"] = max(T * T * pair_stride(-(-nA // ng) * KA * ng_pad(ng))
                      for ng in group_options(nA, L))
    shapes = 0
    for ng in group_options(nA, L):
        for block in (128, 256):
            for G in (1, 4):
                for force in (False, True):
                    replay_pair(N, N, rows, rev, types, M, ng, block, G, force)
                    shapes += 1
    assert shapes == 4 * 2 * 2 * 2


@pytest.mark.parametrize("workload", ["train3", "fcc131k", "bcc2m"])
def test_network_tiles_in_bounds(workload):
    """k_mlp_lds: groups of 64 species-grouped rows (each species padded to
    whole groups, padding -1) taken in runs by a block; every lane's q words
    (the next group's too), the staged w0 / w0^T words and their LDS slots,
    the 16-byte LDS operand reads of both GEMMs and the dU/dq writes, for
    float32 and bf16 whenever the launcher picks this kernel (the LDS image
    within the 160 KB of a gfx950 block and the register arrays large
    enough)."""
    h = synth.WORKLOADS[workload]
    nd = O.num_descriptors(h)
    NN = h["n_neurons"]
    NNp, NDp, NDp32 = (NN + 31) // 32 * 32, (nd + 7) // 8 * 8, (nd + 31) // 32 * 32
    K16 = (nd + 15) // 16 * 16
    KS = K16 // 4
    assert NNp * nd % 4 == 0 and NDp % 8 == 0 and KS % 4 == 0
    G = 64
    SW, ST = K16 + 4, NNp + 4
    SWB, STB = NDp32 + 8, NNp + 8
    assert SW % 4 == 0 and ST % 4 == 0 and SWB % 8 == 0 and STB % 8 == 0   # 16-byte LDS words
    # b0 and w1 (2 N_neu floats) follow the staged weights, 16-byte aligned
    W32 = NNp * SW + K16 * ST                                          # float index
    W16h = (2 * (NNp * SWB + NDp32 * STB) + 15) // 16 * 16 // 2        # half index
    use32 = 4 * (W32 + 2 * NNp) <= 160 * 1024 and KS <= 24             # LDS of a gfx950 block
    use16 = 2 * W16h + 8 * NNp <= 160 * 1024 and NDp32 <= 96
    assert use32 and use16               # every benchmark model runs the LDS kernel
    if not (use32 or use16):
        pytest.skip("the launcher takes the global-memory kernel for this model")
    rng = np.random.default_rng(5)
    for N, T in ((40, 3), (1, 3), (17, 1), (300, 3)):
        types = rng.integers(0, T, N)
        rows_len = (N + G - 1) // G * G + G * T
        rows = []
        for t in range(T):
            idx = [i for i in range(N) if types[i] == t]
            rows += idx + [-1] * ((-len(idx)) % G)
        assert len(rows) <= rows_len
        rows += [-1] * (rows_len - len(rows))
        nets = T
        sizes = dict(q=N * NDp, fp=N * NDp, w0=nets * NNp * nd, w0t=nets * nd * NNp,
                     w0b=nets * NNp * NDp32, w0tb=nets * NDp32 * NNp, rows=rows_len,
                     b0=nets * NNp, w1=nets * NNp, lds32=W32 + 2 * NNp, lds16=W16h + 4 * NNp)
        hi = {k: -1 for k in sizes}

        def touch(k, v):
            hi[k] = max(hi[k], v)
        for base in range(0, rows_len, G):
            first = rows[base]
            if first < 0:
                assert all(r < 0 for r in rows[base:base + G])   # padding groups are whole
                continue
            net = types[first]
            assert all(r < 0 or types[r] == net for r in rows[base:base + G])  # one species
            # staging, one index space of 16-byte words per precision
            nw = NNp * nd // 4
            for k in range(2 * nw):
                if k < nw:
                    touch("w0", net * NNp * nd + 4 * k + 3)
                    for j in range(4):
                        e = 4 * k + j
                        touch("lds32", (e // nd) * SW + e % nd)
                else:
                    touch("w0t", net * nd * NNp + 4 * (k - nw) + 3)
                    r, c = divmod(k - nw, NNp // 4)
                    touch("lds32", NNp * SW + r * ST + 4 * c + 3)
            pad = K16 - nd
            for k in range(NNp * pad):
                touch("lds32", (k // pad) * SW + nd + k % pad)
            for k in range(pad * NNp):
                touch("lds32", NNp * SW + (nd + k // NNp) * ST + k % NNp)
            for k in range(2 * NNp):
                touch("b0" if k < NNp else "w1", net * NNp + k % NNp)
                touch("lds32", W32 + k)
                touch("lds16", W16h + 2 * k + 1)
            c8, t8 = NDp32 // 8, NNp // 8
            n1 = NNp * c8
            for k in range(n1 + NDp32 * t8):
                if k < n1:
                    touch("w0b", net * NNp * NDp32 + 8 * k + 7)
                    r, c = divmod(k, c8)
                    touch("lds16", r * SWB + 8 * c + 7)
                else:
                    touch("w0tb", net * NDp32 * NNp + 8 * (k - n1) + 7)
                    r, c = divmod(k - n1, t8)
                    touch("lds16", NNp * SWB + r * STB + 8 * c + 7)
            for wave in range(4):
                r0 = 16 * wave
                for lane in range(64):
                    col, grp = lane & 15, lane >> 4
                    touch("rows", base + r0 + col)
                    if base + G < rows_len:        # the next group's q words, loaded ahead
                        touch("rows", base + G + r0 + col)
                    atom = rows[base + r0 + col]
                    for v in range(24 // 4):       # float32 q words
                        c = KS * grp + 4 * v
                        if 4 * v < KS and atom >= 0 and c < NDp:
                            touch("q", atom * NDp + c + 3)
                    for s_ in range(24 // 8):      # bf16 q words
                        d0 = 32 * s_ + 8 * grp
                        if 32 * s_ < NDp32 and atom >= 0 and d0 < NDp:
                            touch("q", atom * NDp + d0 + 7)
                    for nb in range(NNp // 16):
                        for off in (0, NNp):             # b0 and w1 of the activation
                            touch("lds32", W32 + off + 16 * nb + 4 * grp + 3)
                            touch("lds16", W16h + 2 * (off + 16 * nb + 4 * grp + 3) + 1)
                        for v in range(KS // 4):
                            touch("lds32", (16 * nb + col) * SW + KS * grp + 4 * v + 3)
                        for s_ in range(NDp32 // 32):
                            touch("lds16", (16 * nb + col) * SWB + 32 * s_ + 8 * grp + 7)
                    dblocks = -(-nd // 16)
                    for db in range(0, dblocks, 2):
                        two = db + 1 < dblocks
                        d0 = 16 * db + col
                        d1 = d0 + 16
                        for nb in range(NNp // 16):
                            for d in ((d0, d1) if two else (d0,)):
                                touch("lds32", NNp * SW + d * ST + 16 * nb + 4 * grp + 3)
                        for p_ in range(NNp // 32):
                            for d in (d0 if d0 < NDp32 else 0, d1 if two and d1 < NDp32 else 0):
                                touch("lds16", NNp * SWB + d * STB + 32 * p_ + 16 + 4 * grp + 3)
                        for r in range(4):
                            touch("rows", base + r0 + 4 * grp + r)
                            at = rows[base + r0 + 4 * grp + r]
                            if at >= 0:
                                for d in ((d0, d1) if two else (d0,)):
                                    if d < nd:
                                        touch("fp", at * NDp + d)
        for k, n in sizes.items():
            if (k == "lds32" and not use32) or (k == "lds16" and not use16):
                continue
            assert hi[k] < n, (N, k, hi[k], n)


def test_cell_rank_sort_emulation():
    """k_cell_sort's wave algorithm, emulated lane by lane: every lane's ranks
    (count of smaller keys over the cell, read 64 at a time) are a
    permutation of 0..n-1 that puts the cell in key order, and every read and
    write stays inside the cell's segment, for cells of 1..1024 atoms (larger
    cells take the one-lane insertion sort)."""
    rng = np.random.default_rng(11)
    per = 16
    for n in (1, 2, 5, 63, 64, 65, 130, 257, 1000, 1024):
        N = 5000
        ext = rng.permutation(N)
        seg = rng.choice(N, size=n, replace=False)
        p = seg.copy()
        keys_lane = {}
        for lane in range(64):
            for a in range(per):
                idx = lane + 64 * a
                if idx < n:
                    keys_lane[(lane, a)] = (p[idx], ext[p[idx]])
        rank = {k: 0 for k in keys_lane}
        for b0 in range(0, n, 64):
            kb = [ext[p[b0 + l]] if b0 + l < n else np.iinfo(np.int32).max for l in range(64)]
            for l in range(min(64, n - b0)):
                for k, (_, key) in keys_lane.items():
                    rank[k] += int(kb[l] < key)
        out = np.full(n, -1)
        for k, (v, _) in keys_lane.items():
            assert 0 <= rank[k] < n
            out[rank[k]] = v
        assert (out >= 0).all()
        assert np.array_equal(out, seg[np.argsort(ext[seg])])


def test_candidate_sequence_steps_reproduce_the_sequential_scan():
    """k_build_rows_wide's sixteen lanes per atom (structures without cells):
    the candidate sequence is taken sixteen at a time (lane s the s-th of each
    step), and the (atom, image) pairs each lane decodes from its sequence
    index, in step and lane order, are those of the sequential scan, inside
    the structure's atoms and image reach (the members' slots then follow from
    the ballot counts emulated below)."""
    G = 16
    for total in (0, 1, 15, 16, 17, 100, 541):
        got = [c0 + s for c0 in range(0, total, G) for s in range(G) if c0 + s < total]
        assert got == list(range(total))
    for reach in ((1, 1, 1), (2, 1, 0), (0, 0, 3), (2, 2, 2)):
        R0, R1, R2 = reach
        start, count = 37, 11
        seq = [(start + j, o0, o1, o2) for j in range(count) for o0 in range(-R0, R0 + 1)
               for o1 in range(-R1, R1 + 1) for o2 in range(-R2, R2 + 1)]
        w1, w2 = 2 * R1 + 1, 2 * R2 + 1
        nimg = (2 * R0 + 1) * w1 * w2
        total = count * nimg
        got = []
        for c0 in range(0, total, G):
            for s_ in range(G):
                c = c0 + s_
                if c >= total:
                    continue
                jl, img = divmod(c, nimg)
                assert 0 <= jl < count
                got.append((start + jl, img // (w1 * w2) - R0, (img // w2) % w1 - R1, img % w2 - R2))
        assert got == seq


def test_cell_build_ballot_placement_emulation():
    """k_build_rows for cell structures, four lanes per atom: a cell's atoms
    are taken four at a time (lane s the (k0 + s)-th), and an accepted one's
    slot is the count so far plus the accepted lanes below it in the same
    step (ballot popcounts).  Emulated lane by lane against a one-lane scan:
    the same row in the same order, and every slot written is below the row
    capacity while the count keeps counting past it."""
    rng = np.random.default_rng(12)
    G = 4
    for trial in range(200):
        ncell = int(rng.integers(1, 28))
        counts = rng.integers(0, 30, ncell)
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
        accept = rng.random(int(counts.sum())) < rng.uniform(0.05, 0.9)
        cap = int(rng.integers(1, 80))
        seq = [int(starts[c] + k) for c in range(ncell) for k in range(counts[c])
               if accept[starts[c] + k]]
        row = [None] * cap
        count = 0
        for c in range(ncell):
            s0, cnt = int(starts[c]), int(counts[c])
            for k0 in range(0, cnt, G):
                take = [k0 + s < cnt and bool(accept[s0 + k0 + s]) for s in range(G)]
                for s in range(G):
                    if take[s]:
                        p = count + sum(take[:s])
                        if p < cap:
                            assert row[p] is None
                            row[p] = s0 + k0 + s
                count += sum(take)
        assert count == len(seq)
        assert row[:min(cap, count)] == seq[:cap]


def test_lockstep_binary_searches_match_one_at_a_time():
    """k_reverse's four searches per lane advance together, each stepping only
    while it has neither found its key nor emptied its range; the positions
    found are those of a plain binary search for the (index, code) key in a
    row sorted by (index, code), and a missing key is reported."""
    rng = np.random.default_rng(13)

    def plain(row, key):
        lo, hi = 0, len(row) - 1
        while lo <= hi:
            mid = (lo + hi) >> 1
            if row[mid] == key:
                return mid
            if row[mid] < key:
                lo = mid + 1
            else:
                hi = mid - 1
        return -1

    for trial in range(300):
        rows, keys = [], []
        for u in range(4):
            n = int(rng.integers(0, 90))
            row = sorted(set((int(rng.integers(0, 500)), int(rng.integers(0, 4)))
                             for _ in range(n)))
            rows.append(row)
            if row and rng.random() < 0.8:
                keys.append(row[int(rng.integers(0, len(row)))])
            else:
                keys.append((int(rng.integers(0, 500)), int(rng.integers(0, 4))))
        lo = [0] * 4
        hi = [len(r) - 1 for r in rows]
        found = [-1] * 4
        steps = 0
        while True:
            live = [found[u] < 0 and lo[u] <= hi[u] for u in range(4)]
            if not any(live):
                break
            steps += 1
            assert steps <= 64
            for u in range(4):
                if not live[u]:
                    continue
                mid = (lo[u] + hi[u]) >> 1
                assert 0 <= mid < len(rows[u])
                if rows[u][mid] == keys[u]:
                    found[u] = mid
                elif rows[u][mid] < keys[u]:
                    lo[u] = mid + 1
                else:
                    hi[u] = mid - 1
        for u in range(4):
            assert found[u] == plain(rows[u], keys[u])
            if keys[u] in rows[u]:
                assert rows[u][found[u]] == keys[u]


def test_row_check_lanes_cover_every_entry_once():
    """k_check_rows with four lanes per atom and four entries per lane at a
    time: lane s of an atom visits entries m0 + 4u (m0 = s, s + 16, ...), so
    the lanes together visit every entry of the row exactly once."""
    G, U = 4, 4
    for nn in range(0, 130):
        seen = []
        for s in range(G):
            for m0 in range(s, nn, U * G):
                for u in range(U):
                    m = m0 + u * G
                    if m < nn:
                        seen.append(m)
        assert sorted(seen) == list(range(nn))
