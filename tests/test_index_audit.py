"""Host replay of the index arithmetic of the particle kernels (no GPU).

The sweep writes a boundary site's post-collision moments through the entry
index kept in the site's record, and the IS substep writes q populations at
element indices of the state layout.  This replays, in numpy, what the
kernels index over 40 steps of the 256^3 workload (500 spheres r = 6, FP32
records, the AA pattern's two layouts alternating) with the spheres moving at
up to 0.03 lu/step per axis, following the kernels' order in the owner-map
mode (balls too large for kind grids): the per-particle sums release the map
and flags at the old shifts, the particle update moves the shifts, the stamp
claims the new ones (lowest entry wins, 2e + [IS]), the prepare pass sets
flags and records, the next sweep reads them.  The kind-grid mode settles
the same owners (lowest particle id among BS/IS claimers); its flags and
owners are compared with the oracle's site kinds on the GPU.  Invariants:
  - every site flagged "owned BS" holds a record whose entry index lies in
    [0, nent) and names a BS entry placed at that very site;
  - every record index the sweep may follow was written by the prepare pass
    of the same step (records start at index -1 and are never cleared);
  - every element an IS write or a shifted pull touches lies inside the
    population array (blocks of 2048 sites holding all 19 populations),
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
    B = 2048  # FP32 populations: blocks of 2048 sites holding all 19
    PS = (NT + B - 1) // B * B

    def elem(i, site):
        return (site // B) * (19 * B) + i * B + site % B
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
                el = elem(i, cc[:, 0] + L[0] * (cc[:, 1] + L[1] * cc[:, 2]))
            else:  # post-collision half: f*_i(x) at [opp(i)][x]
                el = elem(OPP[i], s[is_owned])
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


def test_kind_grid_protocol_sharing_lists_and_flag_changes():
    """The kind-grid mode (balls whose kind grid fits 8192 bytes, as the
    spheres of r = 6 of the 256^3 workload) settles a site's owner from the
    kind grids of the particle and of its sharing list: every particle of the
    box whose centre lay within r_p + r_q + 3 at the start of the step.
    Replayed on the host over 60 steps of a 128^3 box with 30 spheres of
    r = 6 at the workload's spacing, moving at up to 0.03 lu/step per axis,
    and three pairs closing on each other until their balls share sites:
      - every particle whose ball covers one of p's sites after the
        translation, or one of the sites p held before it, is in p's list (so
        the lookups see every claimer);
      - the flag of a site changes only where the prepare pass writes it: at
        the sites, new and old, of a particle whose shift changed;
      - every owned BS site's record names the owner's BS entry at that site.
    Flags: 0 outside every ball, 1 (ball) where some ball covers the site,
    2 where the lowest particle id among the BS and IS claimers has a BS
    entry."""
    L = np.array([128, 128, 128])
    NT = int(np.prod(L))
    r6 = 6.0
    # three pairs 1.5 lu apart at the surface, closing at 0.05 lu/step
    pairs0 = [((30.3, 31.7, 29.2), (1, 0, 0)), ((90.6, 40.1, 70.4), (0, 1, 0)), ((50.2, 95.3, 100.9), (1, 1, 1))]
    xs, us = [], []
    for c, dvec in pairs0:
        dvec = np.asarray(dvec, dtype=np.float64) / np.linalg.norm(dvec)
        xs += [np.asarray(c), np.asarray(c) + (2 * r6 + 1.5) * dvec]
        us += [0.025 * dvec, -0.025 * dvec]
    others = wl.suspension(19, tuple(L), 40, r6, 1.2, seed=23)
    ux = wl.seeded_velocities(40, 3, 0.03, seed=24)
    for j in range(40):
        c = np.asarray(others["x"][j])
        d = np.array(xs) - c
        d -= L * np.floor(d / L + 0.5)
        if np.sqrt((d * d).sum(axis=1)).min() > 2 * r6 + 4.0:
            xs.append(c)
            us.append(ux[j])
        if len(xs) == 30:
            break
    x0 = np.mod(np.array(xs), L)
    u = np.array(us)
    n = len(x0)
    rad = np.full(n, r6)
    b0 = np.floor(x0 + 0.5).astype(np.int64)
    phi = x0 - b0
    offs, kinds, pid = [], [], []
    for j in range(n):
        o, k = template(rad[j], phi[j])
        offs.append(o)
        kinds.append(k)
        pid.append(np.full(len(k), j))
    off = np.concatenate(offs)
    kind = np.concatenate(kinds)
    pid = np.concatenate(pid)
    nent = len(kind)
    e_idx = np.arange(nent)
    x = x0.copy()
    k = np.zeros((n, 3), dtype=np.int64)

    def sites(kk):
        c = np.mod(b0[pid] + kk[pid] + off, L)
        return c[:, 0] + L[0] * (c[:, 1] + L[1] * c[:, 2])

    def truth(s):
        """Flags and the owner entry of owned BS sites for entries at sites s."""
        cover = np.zeros(NT, dtype=bool)
        cover[s] = True
        claim = kind != 3
        own_pid = np.full(NT, n, dtype=np.int64)
        np.minimum.at(own_pid, s[claim], pid[claim])
        bs_own = claim & (own_pid[s] == pid) & (kind == 1)
        flag = cover.astype(np.int8)
        flag[s[bs_own]] = 2
        rec = np.full(NT, -1, dtype=np.int64)
        rec[s[bs_own]] = e_idx[bs_own]
        return flag, rec

    def sharing(xs_):
        d = xs_[:, None, :] - xs_[None, :, :]
        d -= L * np.floor(d / L + 0.5)
        dist = np.sqrt((d * d).sum(axis=2))
        return (dist <= rad[:, None] + rad[None, :] + 3.0) & ~np.eye(n, dtype=bool)

    s = sites(k)
    flag, rec = truth(s)
    shared = 0
    for t in range(60):
        nb = sharing(x)  # centres at the start of the step
        x = x + u
        knew = np.floor(x - x0 + 0.5).astype(np.int64)
        moved = (knew != k).any(axis=1)
        s_old = s
        s = sites(knew)
        # sites covered by two balls at the new shifts: the two know each other
        order = np.argsort(s, kind="stable")
        srt, ps = s[order], pid[order]
        same = (srt[1:] == srt[:-1]) & (ps[1:] != ps[:-1])
        shared += int(same.sum())
        for i_, j_ in zip(ps[1:][same], ps[:-1][same]):
            assert nb[i_, j_] and nb[j_, i_], (t, i_, j_)
        # a site p left, now covered by another ball: that ball is in p's list
        cov_new = np.full(NT, -1, dtype=np.int64)
        cov_new[s] = pid
        q = cov_new[s_old]
        hit = (q >= 0) & (q != pid)
        for i_, j_ in zip(pid[hit], q[hit]):
            assert nb[i_, j_], (t, i_, j_)
        flag_new, rec_new = truth(s)
        # flags change only at the new and old sites of moved particles
        written = np.zeros(NT, dtype=bool)
        mv = moved[pid]
        written[s[mv]] = True
        written[s_old[mv]] = True
        assert not ((flag_new != flag) & ~written).any(), t
        # records: owned BS sites name a BS entry of the owner placed there
        bs_sites = np.flatnonzero(flag_new == 2)
        r = rec_new[bs_sites]
        assert r.min() >= 0 and r.max() < nent and np.all(kind[r] == 1)
        assert np.array_equal(s[r], bs_sites)
        flag, rec, k = flag_new, rec_new, knew
    assert shared > 0
