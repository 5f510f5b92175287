"""CPU model checks of the ILU(0) row form's schedule (k_ilu_up_rows) and
factor layout (IluLayout), written from their definitions in the kernel
source: the anti-diagonal steps d = i + m t within bands of rows or in one
pass with several rows per thread, the LDS ring of the last RING diagonals,
the halo of the band before (rewritten in place), the prefetch buffers with
fixed roles d mod PF, and the layout positions.

These are pure-Python models of the kernel's index arithmetic, not of the
method: they check that the schedule reads every neighbour's final value,
that no LDS entry is read and written by different threads in the same step,
that each step finds its own point in its buffer, and that the layout maps
points to distinct in-range positions.  The GPU tests check the kernel's
values against the oracle."""
import numpy as np
import pytest

GAL = {"M": 3, "RING": 9, "HR": 2, "lo": list(range(12)), "up": [13 + k for k in range(12)], "PF": 3}
FIVE = {"M": 1, "RING": 2, "HR": 1, "lo": [7, 11], "up": [13, 17], "PF": 4}


def bands(ny, NT):
    nb = (ny + NT - 1) // NT
    base, extra = ny // nb, ny % nb
    return nb, (lambda b: b * base + min(b, extra))


def emulate(nx, ny, NT, S, seed):
    rng = np.random.default_rng(seed)
    M, RG, HR = S["M"], S["RING"], S["HR"]
    F = rng.standard_normal((25, ny, nx)) * 0.1
    F[12] = 1.0 + rng.random((ny, nx))
    r = rng.standard_normal((ny, nx))
    # the lexicographic solves, directly
    y = r.copy()
    for j in range(ny):
        for i in range(nx):
            for s in S["lo"]:
                dx, dy = s % 5 - 2, s // 5 - 2
                if 0 <= i + dx < nx and 0 <= j + dy < ny:
                    y[j, i] -= F[s, j, i] * y[j + dy, i + dx]
    z = y.copy()
    for j in reversed(range(ny)):
        for i in reversed(range(nx)):
            for s in S["up"]:
                dx, dy = s % 5 - 2, s // 5 - 2
                if 0 <= i + dx < nx and 0 <= j + dy < ny:
                    z[j, i] -= F[s, j, i] * z[j + dy, i + dx]
            z[j, i] /= F[12, j, i]
    nb, band0 = bands(ny, NT)
    banded = nb > 1
    ring, ringtag = np.full(RG * NT, np.nan), [None] * (RG * NT)
    halo, halotag = np.full(HR * nx, np.nan), [None] * (HR * nx)
    w = r.copy()

    def sweep(fwd):
        for bi in (range(nb) if fwd else reversed(range(nb))):
            j0, R = band0(bi), band0(bi + 1) - band0(bi)
            assert not banded or R >= 3
            nd = (nx - 1) + M * (R - 1) + 1
            for d in (range(nd) if fwd else reversed(range(nd))):
                reads, writes, new = [], [], []
                for t in range(min(R, NT)):
                    i, j = d - M * t, j0 + t
                    if not 0 <= i < nx:
                        continue
                    v = w[j, i]
                    for s in (S["lo"] if fwd else S["up"]):
                        dx, dy = s % 5 - 2, s // 5 - 2
                        if not (0 <= i + dx < nx and 0 <= j + dy < ny):
                            continue
                        if (fwd and t + dy >= 0) or (not fwd and t + dy < R):
                            loc = ("r", ((d + dx + M * dy) % RG) * NT + t + dy)
                            val, tag = ring[loc[1]], ringtag[loc[1]]
                        else:
                            hi = HR + t + dy if fwd else t + dy - R
                            assert 0 <= hi < HR
                            loc = ("h", hi * nx + i + dx)
                            val, tag = halo[loc[1]], halotag[loc[1]]
                        assert tag == (j + dy, i + dx)
                        reads.append((loc, t))
                        v -= F[s, j, i] * val
                    if not fwd:
                        v /= F[12, j, i]
                    new.append((t, i, j, v))
                    writes.append((("r", (d % RG) * NT + t), t))
                    if banded and fwd and t >= R - HR:
                        writes.append((("h", (t - (R - HR)) * nx + i), t))
                    if banded and not fwd and t < HR:
                        writes.append((("h", t * nx + i), t))
                owner = {}
                for loc, t in writes:
                    assert loc not in owner
                    owner[loc] = t
                for loc, t in reads:
                    assert owner.get(loc, t) == t, ("read and written in one step", loc)
                for t, i, j, v in new:
                    k = (d % RG) * NT + t
                    ring[k], ringtag[k] = v, (j, i)
                    h = (t - (R - HR)) * nx + i if fwd else t * nx + i
                    if banded and ((fwd and t >= R - HR) or (not fwd and t < HR)):
                        halo[h], halotag[h] = v, (j, i)
                    w[j, i] = v

    sweep(True)
    np.testing.assert_allclose(w, y, rtol=1e-12, atol=1e-12)
    sweep(False)
    np.testing.assert_allclose(w, z, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", ["gal", "five"])
def test_banded_schedule_reads_final_values_without_races(name):
    S = GAL if name == "gal" else FIVE
    n = 0
    for NT in (4, 5, 8):
        for ny in range(5, 3 * NT + 3):
            for nx in (5, 7, 11):
                nb = (ny + NT - 1) // NT
                if nb > 1 and ny // nb < 3:
                    continue      # the kernel's bands have at least NT / 2 rows
                emulate(nx, ny, NT, S, seed=n)
                n += 1
    assert n > 50


def test_prefetch_buffers_hold_each_steps_point():
    """Step d uses buffer d mod PF and refills it with the point of step
    d + PF (forward) or d - PF (backward); the loops start PF steps early."""
    for M, PF in ((3, 3), (1, 4)):
        for nx in range(5, 14):
            for R in range(1, 12):
                nd = (nx - 1) + M * (R - 1) + 1
                for t in range(R + 3):
                    buf = [None] * PF
                    for d in range(-PF, (nd + PF - 1) // PF * PF):
                        i = d - M * t
                        if t < R and 0 <= i < nx:
                            assert buf[d % PF] == i
                        buf[d % PF] = i + PF
                    buf = [None] * PF
                    top = (nd + PF - 1) // PF * PF
                    for d in range(top + PF - 1, -1, -1):
                        i = d - M * t
                        if d >= top:
                            assert not (t < R and 0 <= i < nx)
                        if t < R and 0 <= i < nx:
                            assert buf[d % PF] == i
                        buf[d % PF] = i - PF


@pytest.mark.parametrize("NT,M,NLO", [(64, 3, 12), (128, 1, 2)])
def test_factor_layout_positions_are_distinct_and_in_range(NT, M, NLO):
    for ny in [5, 17, 63, 64, 65, NT, NT + 1, 2 * NT + 3, 3 * NT - 1]:
        for nx in (5, 9, M * NT, M * NT + 1, M * NT + 7):
            # one band (rows t, t + NT, ... per lane) when nx <= M NT
            if nx <= M * NT:
                nb, j0 = 1, (lambda b: 0 if b == 0 else ny)
            else:
                nb, j0 = bands(ny, NT)
            base, extra = ny // nb, ny % nb
            rmax = base + (1 if extra else 0)
            TS = NT if rmax > NT else (rmax + 63) // 64 * 64
            DT = nb * (nx - M) + M * ny
            size = DT * (2 * NLO + 1) * TS
            assert TS <= NT
            seen, acc = set(), 0
            for b in range(nb):
                d0 = b * (nx - M) + M * j0(b)
                assert d0 == acc
                R = j0(b + 1) - j0(b)
                acc += (nx - 1) + M * (R - 1) + 1
                c = extra * (base + 1)
                for r in range(R):
                    j, t = j0(b) + r, r % NT
                    assert (j // (base + 1) if j < c else extra + (j - c) // base) == b
                    for i in range(nx):
                        dd = d0 + i + M * r
                        pos = [(dd * NLO + k) * TS + t for k in range(NLO)]
                        pos += [(DT * NLO + dd * (NLO + 1) + k) * TS + t for k in range(NLO + 1)]
                        for a in pos:
                            assert 0 <= a < size and a not in seen
                            seen.add(a)
            assert acc == DT and j0(nb) == ny


def emulate_one_pass(nx, ny, NT, S, seed):
    """The one-pass form (nx <= m NT): thread t owns rows t, t + NT, ...; at
    step d it solves the row whose steps contain d, and prefetches for the
    row of step d +- PF, whichever row that is."""
    M, RG, PF = S["M"], S["RING"], S["PF"]
    assert nx <= M * NT < M * ny or ny <= NT
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((25, ny, nx)) * 0.1
    F[12] = 1.0 + rng.random((ny, nx))
    r0 = rng.standard_normal((ny, nx))
    y = r0.copy()
    for j in range(ny):
        for i in range(nx):
            for s in S["lo"]:
                dx, dy = s % 5 - 2, s // 5 - 2
                if 0 <= i + dx < nx and 0 <= j + dy < ny:
                    y[j, i] -= F[s, j, i] * y[j + dy, i + dx]
    z = y.copy()
    for j in reversed(range(ny)):
        for i in reversed(range(nx)):
            for s in S["up"]:
                dx, dy = s % 5 - 2, s // 5 - 2
                if 0 <= i + dx < nx and 0 <= j + dy < ny:
                    z[j, i] -= F[s, j, i] * z[j + dy, i + dx]
            z[j, i] /= F[12, j, i]
    multi = ny > NT

    def locate(d, t):
        q = d - M * t
        k = (q // (M * NT) if q >= 0 else 0) if multi else 0
        r, i = t + k * NT, q - k * M * NT
        return r, i, r < ny and 0 <= i < nx

    nd = (nx - 1) + M * (ny - 1) + 1
    ring, tag = np.full(RG * NT, np.nan), [None] * (RG * NT)
    w = r0.copy()
    for fwd in (True, False):
        bufs = [[None] * PF for _ in range(NT)]
        top = (nd + PF - 1) // PF * PF
        steps = range(-PF, top) if fwd else range(top + PF - 1, -1, -1)
        for d in steps:
            reads, writes, new = [], [], []
            for t in range(NT):
                r, i, act = locate(d, t)
                if act:
                    assert bufs[t][d % PF] == (r, i)
                    v = w[r, i]
                    for s in (S["lo"] if fwd else S["up"]):
                        dx, dy = s % 5 - 2, s // 5 - 2
                        if not (0 <= i + dx < nx and 0 <= r + dy < ny):
                            continue
                        loc = ((d + dx + M * dy) % RG) * NT + (t + dy) % NT
                        assert tag[loc] == (r + dy, i + dx)
                        reads.append((loc, t))
                        v -= F[s, r, i] * ring[loc]
                    if not fwd:
                        v /= F[12, r, i]
                    new.append((t, r, i, v))
                    writes.append(((d % RG) * NT + t, t))
                dn = d + PF if fwd else d - PF
                rn, iN, an = locate(dn, t)
                bufs[t][dn % PF] = (rn, iN) if an else None
            owner = dict((loc, t) for loc, t in writes)
            for loc, t in reads:
                assert owner.get(loc, t) == t, ("read and written in one step", loc)
            for t, r, i, v in new:
                k = (d % RG) * NT + t
                ring[k], tag[k] = v, (r, i)
                w[r, i] = v
        np.testing.assert_allclose(w, y if fwd else z, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", ["gal", "five"])
def test_one_pass_schedule_with_several_rows_per_thread(name):
    S = GAL if name == "gal" else FIVE
    n = 0
    for NT in (4, 6, 8, 10):
        for nx in range(5, S["M"] * NT + 1, 2):
            for ny in (NT + 1, 2 * NT + 3, 3 * NT):
                if ny < 5:
                    continue
                emulate_one_pass(nx, ny, NT, S, seed=n)
                n += 1
    assert n > 5
