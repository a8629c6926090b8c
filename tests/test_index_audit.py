"""Host replay of the index arithmetic of the particle kernels (no GPU).

The sweep writes a boundary site's post-collision moments through the entry
index kept in the site's record, and the IS substep writes q populations at
element indices of the state layout.  This replays, in numpy, what the
kernels index over 40 steps of the 256^3 workload (500 spheres r = 6, FP32
records, the AA pattern's two layouts alternating) with the spheres moving at
up to 0.03 lu/step per axis, following the kernels' order: the per-particle
sums release the map and flags at the old shifts, the particle update moves
the shifts, the stamp claims the new ones (lowest entry wins, 2e + [IS]), the
prepare pass sets flags and records, the next sweep reads them.  Invariants:
  - every site flagged "owned BS" holds a record whose entry index lies in
    [0, nent) and names a BS entry placed at that very site;
  - every record index the sweep may follow was written by the prepare pass
    of the same step (records start at index -1 and are never cleared);
  - every element an IS write or a shifted pull touches lies below q x PS,
    every site below NT;
  - the releases of a step clear exactly what the previous step set.
This is the arithmetic of the kernels restated on the host; it checks the
design of the flag/record protocol, not the compiled code.
"""
import numpy as np

from paper_1105_2904_amd import workloads as wl

Q19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
OPP = np.array([int(np.flatnonzero((Q19 == -c).all(axis=1))[0]) for c in Q19])
EMPTY = 0x7FFFFFFF


def template(r, phi):
    """Offsets (z, y, x order) and kinds (1 BS, 2 IS, 3 interior) of a ball."""
    R = int(np.ceil(r)) + 1
    g = np.arange(-R - 1, R + 2)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    inside = (X - phi[0]) ** 2 + (Y - phi[1]) ** 2 + (Z - phi[2]) ** 2 <= r * r

    def shifted(a, c):
        return np.roll(a, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))

    bs = inside & np.any([~shifted(inside, c) for c in Q19[1:]], axis=0)
    isb = inside & ~bs & np.any([shifted(bs, c) for c in Q19[1:]], axis=0)
    kind = np.where(bs, 1, np.where(isb, 2, 3))
    sel = inside & (np.abs(Z) <= R) & (np.abs(Y) <= R) & (np.abs(X) <= R)
    return np.stack([X[sel], Y[sel], Z[sel]], axis=1), kind[sel]


def test_flag_record_protocol_and_index_ranges():
    cfg = wl.spheres_3d_config()
    p = cfg["particles"]
    n = len(p["radius"])
    L = np.array(cfg["box"])
    NT = int(np.prod(L))
    PS = (NT + 255) // 256 * 256 + 256
    x0 = np.array(p["x"], dtype=np.float64)
    b0 = np.floor(x0 + 0.5).astype(np.int64)
    phi = x0 - b0
    offs, kinds, pid = [], [], []
    for j in range(n):
        o, k = template(p["radius"][j], phi[j])
        offs.append(o)
        kinds.append(k)
        pid.append(np.full(len(k), j))
    off = np.concatenate(offs)
    kind = np.concatenate(kinds)
    pid = np.concatenate(pid)
    nent = len(kind)
    assert nent < 2 ** 29
    u = wl.seeded_velocities(n, 3, 0.03, seed=12)
    x = x0.copy()
    k = np.zeros((n, 3), dtype=np.int64)

    def sites(kk):
        c = np.mod(b0[pid] + kk[pid] + off, L)
        s = c[:, 0] + L[0] * (c[:, 1] + L[1] * c[:, 2])
        assert s.min() >= 0 and s.max() < NT
        return s, c

    own = np.full(NT, EMPTY, dtype=np.int64)
    flag = np.zeros(NT, dtype=np.int8)
    rec = np.full(NT, -1, dtype=np.int64)
    e_idx = np.arange(nent)
    claim = kind != 3

    def stamp(s):
        np.minimum.at(own, s[claim], 2 * e_idx[claim] + (kind[claim] == 2))

    def prepare(s, c, layout):
        o = own[s]
        flag[s] = np.where((o != EMPTY) & (o % 2 == 0), 2, 1)
        mine = o == 2 * e_idx
        rec[s[mine]] = e_idx[mine]
        is_owned = o == 2 * e_idx + 1
        for i in range(19):
            if layout == "stream":  # post-propagation half: f*_i(x) at [i][x + c_i]
                cc = np.mod(c[is_owned] + Q19[i], L)
                el = i * PS + cc[:, 0] + L[0] * (cc[:, 1] + L[1] * cc[:, 2])
            else:  # post-collision half: f*_i(x) at [opp(i)][x]
                el = OPP[i] * PS + s[is_owned]
            assert el.min() >= 0 and el.max() < 19 * PS

    s, c = sites(k)
    stamp(s)
    prepare(s, c, "stream")
    moved = 0
    for t in range(40):
        # the sweep: every owned-BS flag has a live record naming a BS entry at the site
        bs_sites = np.flatnonzero(flag == 2)
        r = rec[bs_sites]
        assert r.min() >= 0 and r.max() < nent
        assert np.all(kind[r] == 1)
        assert np.array_equal(sites(k)[0][r], bs_sites)
        # per-particle sums: release at the old shifts
        flag[s] = 0
        own[s[claim]] = EMPTY
        assert not flag.any() and np.all(own == EMPTY)
        # particle update and translation (the forces do not matter here)
        x += u
        knew = np.floor(x - x0 + 0.5).astype(np.int64)
        moved += int((knew != k).any(axis=1).sum())
        k = knew
        s, c = sites(k)
        stamp(s)
        prepare(s, c, "swap" if t % 2 == 0 else "stream")
    assert moved > 100
