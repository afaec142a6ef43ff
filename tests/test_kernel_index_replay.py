"""CPU replay of the row kernels' memory accesses on the exact device layouts (no GPU).

The sparse row kernels (SELL-64 with one row per lane, CSR with G lanes per row) issue their
index, value and gather loads before they know which slots of a chunk are real entries, so every slot
must point at valid memory. This module restates the layouts the library packs (slices of 64 rows padded
to their longest row, 16-bit column offsets from a scaled diagonal when every column fits, lane groups
for long coarse rows) and the index arithmetic of the row kernels, lane by lane with numpy, and checks
on the matrices of real hierarchies that

  * every index and value load stays inside the stored arrays,
  * every gather stays inside the gathered vector,
  * the sums over the real entries equal the oracle's product: bit for bit with one lane per row (entry
    order), to rounding with lane groups (lane j sums entries j, j + G, ..., then a fixed butterfly);
  * the prolongations' unit-row layout (a C point's row stores no entry) loads and gathers in range and
    gives the plain layout's bits;
  * the slice-diagonal layout (one column offset per slot of 64 rows, no per-entry columns) is chosen where
    the library's rule takes it, reads its offsets, values and gathers in range (chunks of eight slots and
    one exact rest), and gives the plain layout's bits;
  * both forms of the unit-row prolongation kernel (one lane per row; a wavefront per pair of slices, F
    rows first) load, gather and write in range and give the same bits.

A model of the unit-row kernel that reads the layout as plain SELL-64 (its masks not reaching the kernel)
must show out-of-range gathers, so the replay can tell the two apart.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import CSR, config_system, varcoef3d

SELL_C = 64
BLK = 256
U = 4
COL_SHIFT = 20


@pytest.fixture(scope="module")
def namg():
    import paper_2112_14681_amd as m

    return m


# --------------------------------------------------------------------------------------- layouts
def diag_mul(nrows, ncols):
    return (ncols << COL_SHIFT) // nrows if nrows > 0 else 0


def diag_base(rows, mul):
    return (rows.astype(np.int64) * mul) >> COL_SHIFT


def choose_group(nrows, nnz, lane_entries=8, sell_min_rows=1 << 17):
    avg = nnz / nrows if nrows > 0 else 0.0
    if avg <= 10.0 or nrows >= sell_min_rows:
        return 1
    g = 2
    while g < 64 and g * lane_entries < avg:
        g <<= 1
    return g


class Layout:
    """The device layout of one CSR matrix (nrows x ncols), as the library packs it."""

    def __init__(self, rp, ci, vals, ncols, force_group=0):
        self.nrows = len(rp) - 1
        self.ncols = ncols
        self.mul = diag_mul(self.nrows, ncols)
        rows = np.repeat(np.arange(self.nrows), np.diff(rp))
        off = ci.astype(np.int64) - diag_base(rows, self.mul)
        self.narrow = bool(off.size == 0 or (off.min() >= -32768 and off.max() <= 32767))
        self.group = force_group or choose_group(self.nrows, int(rp[-1]))
        if self.group > 1:
            self.ptr = rp.astype(np.int64)
            self.idx = (off if self.narrow else ci).astype(np.int64)
            self.val = vals.copy()
            return
        lens = np.diff(rp)
        nsl = (self.nrows + SELL_C - 1) // SELL_C
        padded = np.zeros(nsl * SELL_C, np.int64)
        padded[: self.nrows] = lens
        width = padded.reshape(nsl, SELL_C).max(axis=1)
        self.ptr = np.zeros(nsl + 1, np.int64)
        np.cumsum(width * SELL_C, out=self.ptr[1:])
        stored = int(self.ptr[-1])
        self.idx = np.zeros(max(stored, 1), np.int64)  # padding: offset 0 or column 0
        self.val = np.zeros(max(stored, 1))
        k_in_row = np.arange(rp[-1]) - np.repeat(rp[:-1], lens)
        dst = self.ptr[rows // SELL_C] + SELL_C * k_in_row + (rows % SELL_C)
        self.idx[dst] = off if self.narrow else ci
        self.val[dst] = vals
        self.stored = stored


class UnitLayout:
    """The unit-row SELL layout of a prolongation, as the library packs it: the rows of C points (cf == 1)
    store nothing (each must be the unit vector of its coarse index, the number of C points before it, else
    `ok` is False and the plain layout is used); within slice s the l-th F row keeps entry k at
    ptr[s] + k m_s + l, padded to the slice's longest F row."""

    def __init__(self, rp, ci, vals, ncols, cf):
        self.nrows = len(rp) - 1
        self.ncols = ncols
        self.mul = diag_mul(self.nrows, ncols)
        rows = np.repeat(np.arange(self.nrows), np.diff(rp))
        off = ci.astype(np.int64) - diag_base(rows, self.mul)
        self.narrow = bool(off.size == 0 or (off.min() >= -32768 and off.max() <= 32767))
        self.group = 1
        lens = np.diff(rp)
        unit = np.asarray(cf) == 1
        nunits = int(unit.sum())
        first = rp[:-1][unit]
        self.ok = (nunits > 0 and bool(np.all(lens[unit] == 1)) and bool(np.all(vals[first] == 1.0))
                   and bool(np.array_equal(ci[first], np.arange(nunits))))
        nsl = (self.nrows + SELL_C - 1) // SELL_C
        upad = np.zeros(nsl * SELL_C, bool)
        upad[: self.nrows] = unit
        bits = upad.reshape(nsl, SELL_C)
        self.mask_bits = bits
        self.before = np.concatenate([[0], np.cumsum(bits.sum(axis=1))[:-1]]).astype(np.int64)
        lpad = np.zeros(nsl * SELL_C, np.int64)
        lpad[: self.nrows] = np.where(unit, 0, lens)
        expl = np.zeros(nsl * SELL_C, bool)
        expl[: self.nrows] = ~unit
        self.count = expl.reshape(nsl, SELL_C).sum(axis=1).astype(np.int64)
        width = lpad.reshape(nsl, SELL_C).max(axis=1)
        self.ptr = np.zeros(nsl + 1, np.int64)
        np.cumsum(width * self.count, out=self.ptr[1:])
        stored = int(self.ptr[-1])
        self.stored = stored
        self.idx = np.zeros(max(stored, 1), np.int64)
        self.val = np.zeros(max(stored, 1))
        # rank of each explicit row among its slice's explicit rows
        rank = np.cumsum(expl.reshape(nsl, SELL_C), axis=1).reshape(-1)[: self.nrows] - 1
        er = ~unit[rows]
        k_in_row = np.arange(rp[-1]) - np.repeat(rp[:-1], lens)
        dst = self.ptr[rows // SELL_C] + k_in_row * self.count[rows // SELL_C] + rank[rows]
        self.idx[dst[er]] = (off if self.narrow else ci)[er]
        self.val[dst[er]] = vals[er]


def dia_cap(longest_row):
    return 2 * longest_row + 8


class DiaLayout:
    """The slice-diagonal layout of a matrix, as the library packs it, and the library's rule for taking it
    (`use(val_bytes)`): rows with strictly increasing columns, no slice whose union of offsets (column - the
    row's scaled diagonal base) exceeds dia_cap(its longest row), and fewer bytes than SELL-64 (slots x 64 x
    value bytes + 4 per slot against SELL-64's stored entries x (value + column bytes)). Slice s keeps its union in increasing order:
    slot k's entries at ptr[s] + 64 k, its offset at off[1 + ptr[s] / 64 + k]; off[0] is ncols - 1."""

    def __init__(self, rp, ci, vals, ncols):
        rp = np.asarray(rp, np.int64)
        ci = np.asarray(ci, np.int64)
        self.nrows = n = len(rp) - 1
        self.ncols = ncols
        self.mul = diag_mul(n, ncols)
        lens = np.diff(rp)
        rows = np.repeat(np.arange(n), lens)
        off = ci - diag_base(rows, self.mul)
        nsl = (n + SELL_C - 1) // SELL_C
        same_row = rows[1:] == rows[:-1]
        self.sorted = bool(np.all(ci[1:][same_row] > ci[:-1][same_row]))
        sl = rows >> 6
        key = np.unique(sl * (1 << 33) + (off + (1 << 32)))
        ksl = key >> 33
        koff = (key & ((1 << 33) - 1)) - (1 << 32)
        width = np.bincount(ksl, minlength=nsl)
        lpad = np.zeros(nsl * SELL_C, np.int64)
        lpad[:n] = lens
        self.longest = lpad.reshape(nsl, SELL_C).max(axis=1) if nsl else np.zeros(0, np.int64)
        self.width = width
        self.ptr = np.zeros(nsl + 1, np.int64)
        np.cumsum(width * SELL_C, out=self.ptr[1:])
        self.stored = int(self.ptr[-1])
        self.sell_stored = int((self.longest * SELL_C).sum())
        # offsets: slice by slice in increasing order (np.unique sorted the keys that way)
        self.off = np.concatenate([[ncols - 1], koff]).astype(np.int64)
        self.val = np.zeros(max(self.stored, 1))
        # the slot of each entry: its rank among its slice's offsets
        first = np.searchsorted(ksl, np.arange(nsl))
        slot = np.searchsorted(key, sl * (1 << 33) + (off + (1 << 32))) - first[sl]
        self.val[self.ptr[sl] + slot * SELL_C + (rows & 63)] = vals
        self.narrow = bool(off.size == 0 or (off.min() >= -32768 and off.max() <= 32767))

    def use(self, val_bytes, group=1):
        if not (group == 1 and self.sorted and self.nrows > 0):
            return False
        if np.any(self.width > dia_cap(self.longest)):
            return False
        sell = self.sell_stored * (val_bytes + (2 if self.narrow else 4))
        dia = self.stored * val_bytes + 4 * (self.stored // SELL_C + 1)
        return dia < sell


class DiaAccess:
    """Range checks of the slice-diagonal kernels' reads: offsets, values, gathers."""

    def __init__(self, L):
        self.L = L
        self.bad = {"offsets": 0, "values": 0, "gathers": 0}

    def offset(self, i):
        self.bad["offsets"] += int(np.count_nonzero((i < 0) | (i >= len(self.L.off))))
        return self.L.off[np.clip(i, 0, len(self.L.off) - 1)]

    def value(self, k):
        n = max(self.L.stored, 1)
        self.bad["values"] += int(np.count_nonzero((k < 0) | (k >= n)))
        return self.L.val[np.clip(k, 0, n - 1)]

    def gather(self, x, c):
        self.bad["gathers"] += int(np.count_nonzero((c < 0) | (c >= self.L.ncols)))
        return x[np.clip(c, 0, self.L.ncols - 1)]

    def clean(self):
        return all(v == 0 for v in self.bad.values())


def _dia_exact_chunks(w):
    """The chunks dia_row_from walks for a row of w slots: eights, then one chunk of exactly the rest."""
    j, out = 0, []
    while j + 8 <= w:
        out.append((j, 8))
        j += 8
    if w - j > 0:
        out.append((j, w - j))
    return out


def replay_dia_exact(L, x):
    """dia_dot in its exact-chunk form (one row per lane, a wavefront per slice): every chunk's slots exist, so
    offsets and values are read inside the slice; every product is added, padding (value 0) included."""
    a = DiaAccess(L)
    cmax = int(a.offset(np.array([0]))[0])
    acc = np.zeros(L.nrows)
    for s in range(len(L.ptr) - 1):
        rows = np.arange(s * SELL_C, min(L.nrows, (s + 1) * SELL_C), dtype=np.int64)
        lane = rows & 63
        p0, p1 = int(L.ptr[s]), int(L.ptr[s + 1])
        w = (p1 - p0) >> 6
        part = np.zeros(rows.size)
        for j, k in _dia_exact_chunks(w):
            for u in range(k):
                o = int(a.offset(np.array([1 + (p0 >> 6) + j + u]))[0])
                v = a.value(p0 + (j + u) * SELL_C + lane)
                part = part + v * a.gather(x, np.clip(diag_base(rows, L.mul) + o, 0, cmax))
        acc[rows] = part
    return acc, a


def replay_dia_pairs(L, x):
    """k_neumann_pairs's row sums (FP32 square slice-diagonal triangles, two rows per lane): a wavefront takes
    slices 2w and 2w + 1 (lanes 0-31 and 32-63) and lane h of a half rows 2h and 2h + 1 of its slice. When both
    slices hold 64 rows and have the same width, slot k's two values are one 8-byte read at ptr + 64 k + 2h
    and the two gathers one 8-byte read at the pair's first column clamped into [0, cmax - 1], from which a
    select gives x[clamp(r + o)] and x[clamp(r + 1 + o)]; otherwise each row runs alone on its own slice's
    pointers and offsets. Every row sums its slice's slots in slot order, padding included."""
    a = DiaAccess(L)
    n, nsl = L.nrows, len(L.ptr) - 1
    cmax = int(a.offset(np.array([0]))[0])
    acc = np.zeros(n)
    for sA in range(0, nsl, 2):
        if (sA + 2) * SELL_C <= n and (int(L.ptr[sA + 1]) - int(L.ptr[sA])) == (int(L.ptr[sA + 2]) - int(L.ptr[sA + 1])):
            w = (int(L.ptr[sA + 1]) - int(L.ptr[sA])) >> 6
            for s in (sA, sA + 1):
                p = int(L.ptr[s])
                h = np.arange(32, dtype=np.int64)
                r = s * SELL_C + 2 * h
                s0, s1 = np.zeros(32), np.zeros(32)
                for j, k in _dia_exact_chunks(w):
                    for u in range(k):
                        o = int(a.offset(np.array([1 + (p >> 6) + j + u]))[0])
                        vi = p + (j + u) * SELL_C + 2 * h
                        v0, v1 = a.value(vi), a.value(vi + 1)
                        c = r + o
                        cc = np.clip(c, 0, cmax - 1)
                        g0, g1 = a.gather(x, cc), a.gather(x, cc + 1)
                        s0 = s0 + v0 * np.where(c >= cmax, g1, g0)
                        s1 = s1 + v1 * np.where(c < 0, g0, g1)
                acc[r], acc[r + 1] = s0, s1
        else:
            for row in range(sA * SELL_C, min(n, (sA + 2) * SELL_C)):
                s = row >> 6
                p0 = int(L.ptr[s])
                w = (int(L.ptr[s + 1]) - p0) >> 6
                t = 0.0
                for k in range(w):
                    o = int(a.offset(np.array([1 + (p0 >> 6) + k]))[0])
                    t = t + float(a.value(np.array([p0 + k * SELL_C + (row & 63)]))[0]) * float(
                        a.gather(x, np.array([min(max(row + o, 0), cmax)]))[0])
                acc[row] = t
    return acc, a


def replay_prolong_unit_rows(L, e, U=U):
    """prolong_unit_rows's loads and gathers, row by row (a thread's second row, in FP32, runs the same index
    stream): an F row walks its slots in chunks of U (4, or 8 where F rows average more than four entries);
    a C point's row takes a virtual first entry (column = C points before it, value 1) in its one chunk,
    whose loads follow the slots of the F row of rank `below` (columns clamped into range, not added).
    Returns P e and the access record."""
    a = Access(L)
    row = np.arange(L.nrows, dtype=np.int64)
    s, lane = row >> 6, row & 63
    bits = L.mask_bits
    is_unit = bits.reshape(-1)[row]
    below = np.cumsum(bits, axis=1).reshape(-1)[row] - is_unit  # C points before this lane in its slice
    mm = L.count[s]
    m = np.maximum(mm, 1)
    p0, lim = L.ptr[s], L.ptr[s + 1]
    k = p0 + np.where(is_unit, np.where(mm > 0, np.minimum(below, mm - 1), 0), lane - below)
    end = np.where(is_unit, p0, lim)
    cu = L.before[s] + below
    base = diag_base(row, L.mul) if L.narrow else np.zeros_like(row)
    virt = is_unit.copy()
    acc = np.zeros(L.nrows)
    while True:
        act = virt | (k < end)
        if not act.any():
            break
        kb = np.where(k < lim, k, np.where(lim > 0, lim - 1, 0))
        oks, cs, vs = [], [], []
        for q in range(U):
            kk = np.where(k + q * m < lim, k + q * m, kb)
            ok = k + q * m < end
            i, v = a.load(kk[act])
            col = base[act] + i if L.narrow else i
            c = np.clip(col, 0, L.ncols - 1)  # a slot that is not this row's decodes another row's offset
            if q == 0:
                va = virt[act]
                ok = ok.copy()
                ok[act] = ok[act] | va
                c = np.where(va, cu[act], c)
                v = np.where(va, 1.0, v)
            oks.append(ok[act])
            cs.append(c)
            vs.append(v)
        xs = [a.gather(e, c) for c in cs]
        part = acc[act]
        for q in range(U):
            part = np.where(oks[q], part + vs[q] * xs[q], part)
        acc[act] = part
        virt[:] = False
        k = k + U * m
    return acc, a


def replay_prolong_unit_pairs(L, e, U=U):
    """prolong_unit_pairs, wavefront by wavefront: a wavefront takes slices 2w and 2w + 1; its lanes take the
    pair's F rows (slice 2w's in rank order, then slice 2w + 1's), 64 at a time, then its C points' rows the
    same way; a lane's row comes from the table the wavefront builds from the two masks. An F row of rank l in
    slice q walks slots ptr + k m_q + l in chunks of U up to the pair's widest F row; a slot past its own end
    loads the pair's first stored slot (a slice with F rows and entries), its column clamped into range, and
    adds 0 times the gathered element. A C point of rank l in slice q reads e[before_q + l]. Returns P e (the
    amount each row adds to x) and the access record; also checks the table's indices and every row written."""
    a = Access(L)
    acc = np.zeros(L.nrows)
    written = np.zeros(L.nrows, np.int64)
    nsl = len(L.ptr) - 1
    lane = np.arange(SELL_C, dtype=np.int64)
    a.bad_table = 0
    for s0 in range(0, nsl, 2):
        qs = [q for q in (0, 1) if s0 + q < nsl]
        um = [L.mask_bits[s0 + q] if q in qs else np.zeros(SELL_C, bool) for q in (0, 1)]
        m = [int(L.count[s0 + q]) if q in qs else 0 for q in (0, 1)]
        p = [int(L.ptr[s0 + q]) if q in qs else 0 for q in (0, 1)]
        w = [(int(L.ptr[s0 + q + 1]) - p[q]) // m[q] if q in qs and m[q] > 0 else 0 for q in (0, 1)]
        nr = [min(SELL_C, L.nrows - (s0 + q) * SELL_C) if q in qs else 0 for q in (0, 1)]
        nc = [int(um[q][: nr[q]].sum()) for q in (0, 1)]
        before = [int(L.before[s0 + q]) if q in qs else 0 for q in (0, 1)]
        ftab = np.full(2 * SELL_C, -1, np.int64)
        ctab = np.full(2 * SELL_C, -1, np.int64)
        for q in (0, 1):
            live = lane < nr[q]
            isc = um[q] & live
            isf = ~um[q] & live
            crank = np.cumsum(um[q]) - um[q]
            frank = np.cumsum(~um[q]) - (~um[q])
            ci_ = q * nc[0] + crank[isc]
            fi_ = q * m[0] + frank[isf]
            a.bad_table += int(np.count_nonzero((ci_ < 0) | (ci_ >= 2 * SELL_C)))
            a.bad_table += int(np.count_nonzero((fi_ < 0) | (fi_ >= 2 * SELL_C)))
            ctab[np.clip(ci_, 0, 2 * SELL_C - 1)] = q * SELL_C + lane[isc]
            ftab[np.clip(fi_, 0, 2 * SELL_C - 1)] = q * SELL_C + lane[isf]
        row0 = s0 * SELL_C
        nf = m[0] + m[1]
        wmax = max(w[0] if m[0] > 0 else 0, w[1] if m[1] > 0 else 0)
        safe = p[0] if (m[0] > 0 and w[0] > 0) else p[1]
        for f0 in range(0, nf, SELL_C):
            f = f0 + lane
            act = f < nf
            second = f >= m[0]
            rank = np.where(second, f - m[0], f)
            mq = np.where(second, m[1], m[0])
            pq = np.where(second, p[1], p[0])
            wl = np.where(act, np.where(second, w[1], w[0]), 0)
            pos = np.where(act, ftab[np.clip(f, 0, 2 * SELL_C - 1)], 0)
            a.bad_table += int(np.count_nonzero(act & (pos < 0)))
            row = row0 + pos
            base = diag_base(row, L.mul) if L.narrow else np.zeros_like(row)
            part = np.zeros(SELL_C)
            for k in range(0, wmax, U):
                for u in range(U):
                    ok = k + u < wl
                    kk = np.where(ok, pq + (k + u) * mq + rank, safe)
                    i, v = a.load(kk)
                    col = base + i if L.narrow else i
                    c = np.clip(col, 0, L.ncols - 1)
                    ev = a.gather(e, c)
                    part = part + np.where(ok, v, 0.0) * ev
            rows = row[act]
            written[rows] += 1
            acc[rows] = part[act]
        ncp = nc[0] + nc[1]
        for c0 in range(0, ncp, SELL_C):
            c = c0 + lane
            act = c < ncp
            second = c >= nc[0]
            col = np.where(second, before[1] + (c - nc[0]), before[0] + c)[act]
            pos = ctab[np.clip(c, 0, 2 * SELL_C - 1)][act]
            a.bad_table += int(np.count_nonzero(pos < 0))
            rows = row0 + pos
            written[rows] += 1
            acc[rows] = 0.0 + 1.0 * a.gather(e, col)
    a.bad_rows = int(np.count_nonzero(written != 1))  # every row written exactly once
    return acc, a


class Access:
    """Collects every index/value load position and every gather column; checks their ranges."""

    def __init__(self, layout):
        self.L = layout
        self.bad_loads = 0
        self.bad_gathers = 0

    def load(self, kk):
        n_store = len(self.L.val) if self.L.group > 1 else max(self.L.stored, 1)
        self.bad_loads += int(np.count_nonzero((kk < 0) | (kk >= n_store)))
        return self.L.idx[np.clip(kk, 0, n_store - 1)], self.L.val[np.clip(kk, 0, n_store - 1)]

    def gather(self, x, c):
        self.bad_gathers += int(np.count_nonzero((c < 0) | (c >= self.L.ncols)))
        return x[np.clip(c, 0, self.L.ncols - 1)]


# ------------------------------------------------------------------------------- kernel replays
def replay_one_row_per_lane(L, x):
    """SELL-64 with one row per lane (8-byte values), or CSR with G lanes per row: row_dot_impl."""
    acc_all = np.zeros(L.nrows)
    a = Access(L)
    G = L.group
    nthreads = ((L.nrows * G + BLK - 1) // BLK) * BLK
    g = np.arange(nthreads, dtype=np.int64)
    row, sub = g // G, g % G
    live = row < L.nrows
    row, sub = row[live], sub[live]
    step = SELL_C if G == 1 else G
    if G == 1:
        k = L.ptr[row >> 6] + (row & 63)
        end = L.ptr[(row >> 6) + 1]
    else:
        k = L.ptr[row] + sub
        end = L.ptr[row + 1]
    base = diag_base(row, L.mul) if L.narrow else np.zeros_like(row)
    acc = np.zeros(row.size)
    while True:
        act = k < end
        if not act.any():
            break
        kk_list, ok_list = [], []
        for u in range(U):
            ok = act & (k + u * step < end)
            kk = np.where(ok, k + u * step, k)
            kk_list.append(kk[act])
            ok_list.append(ok[act])
        cols, vals = [], []
        for kk in kk_list:
            i, v = a.load(kk)
            cols.append(base[act] + i if L.narrow else i)
            vals.append(v)
        xs = [a.gather(x, c) for c in cols]
        part = acc[act]
        for u in range(U):
            part = np.where(ok_list[u], part + vals[u] * xs[u], part)
        acc[act] = part
        k = k + U * step
    if G == 1:
        acc_all[row] = acc
    else:
        # the xor butterfly over the group: lanes j and j ^ off pair up, in a fixed order
        s = acc.reshape(-1, G)
        off = G // 2
        while off > 0:
            s = s + s[:, np.arange(G) ^ off]
            off //= 2
        acc_all[row.reshape(-1, G)[:, 0]] = s[:, 0]
    return acc_all, a


# -------------------------------------------------------------------------------- the matrices
def strict_part(rp, ci, vals, lower):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    keep = ci < rows if lower else ci > rows
    cnt = np.bincount(rows[keep], minlength=len(rp) - 1)
    nrp = np.zeros(len(rp), np.int64)
    np.cumsum(cnt, out=nrp[1:])
    return nrp, ci[keep], vals[keep]


def hierarchy_operators(namg, A, **kw):
    """Every operator a V-cycle multiplies with, as (name, rowptr, colind, vals, ncols, force_group, cf); cf is
    the level's C/F splitting for a prolongation, else None."""
    H = namg.Hierarchy(A, device=-1, **kw)
    info = H.info()
    ops = []
    for l in range(info["levels"] - 1):
        e = H.export_level(l)
        Arp, Aci, Av = e["A"]
        n = len(Arp) - 1
        ops.append((f"A{l}", Arp, Aci, Av, n, 0, None))
        if l == 0:
            ops.append(("A0 fp64", Arp, Aci, Av, n, 1, None))
        Prp, Pci, Pv, nc = e["P"]
        ops.append((f"P{l}", Prp, Pci, Pv, nc, 0, e["cf"]))
        R = sp.csr_matrix((Pv, Pci, Prp), shape=(n, nc)).T.tocsr()
        R.sort_indices()
        ops.append((f"R{l}", R.indptr, R.indices, R.data, n, 0, None))
        for lower in (True, False):
            rp, ci, v = strict_part(Arp, Aci, Av, lower)
            ops.append((f"A{l} {'lower' if lower else 'upper'}", rp, ci, v, n, 0, None))
        if l == 0 and kw.get("ilu_levels", 1) != 0:
            f = H.export_ilu(0)
            ops.append(("ILU L_s", *f["L"], n, 0, None))
            ops.append(("ILU U_s", *f["U"], n, 0, None))
    H.close()
    return ops


def _systems():
    yield "varcoef 33^3", varcoef3d(33, 0.5, 1001)[0]
    yield "varcoef 47^3 stretched", varcoef3d(47, 1.0, 1002, 100.0)[0]
    yield "varcoef 65^3", varcoef3d(65, 0.5, 1003)[0]
    yield "permuted 34^3", config_system("c4r", 34)[0]


@pytest.mark.parametrize("case", range(4))
def test_row_kernel_accesses_in_range(namg, case):
    name, A = list(_systems())[case]
    rng = np.random.default_rng(case)
    dia_used, pairs_used = set(), set()
    for label, rp, ci, v, ncols, fg, cf in hierarchy_operators(namg, A):
        L = Layout(np.asarray(rp), np.asarray(ci), np.asarray(v), ncols, fg)
        x = rng.standard_normal(ncols)
        y, acc = replay_one_row_per_lane(L, x)
        assert acc.bad_loads == 0 and acc.bad_gathers == 0, (name, label, "one row per lane", acc.bad_loads,
                                                              acc.bad_gathers)
        if ncols == len(rp) - 1 and L.group == 1:  # one lane per row sums in entry order: the oracle's bits
            ref = O.spmv(CSR(ncols, np.asarray(rp, np.int32), np.asarray(ci, np.int32), np.asarray(v)), x)
            assert np.array_equal(y, ref), (name, label)
        else:
            ref = sp.csr_matrix((v, ci, rp), shape=(len(rp) - 1, ncols)) @ x
            np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)
        if cf is not None:
            Lu = UnitLayout(np.asarray(rp), np.asarray(ci), np.asarray(v), ncols, cf)
            assert Lu.ok, (name, label)  # a C/F splitting's P always has the unit-row form
            assert Lu.stored < L.stored, (name, label)
            for unroll in (4, 8):
                yu, accu = replay_prolong_unit_rows(Lu, x, unroll)
                assert accu.bad_loads == 0 and accu.bad_gathers == 0, (name, label, "unit rows", unroll,
                                                                      accu.bad_loads, accu.bad_gathers)
                yp, accp = replay_prolong_unit_pairs(Lu, x, unroll)
                assert accp.bad_loads == 0 and accp.bad_gathers == 0, (name, label, "unit pairs", unroll,
                                                                      accp.bad_loads, accp.bad_gathers)
                assert accp.bad_table == 0 and accp.bad_rows == 0, (name, label, "unit pairs", unroll,
                                                                    accp.bad_table, accp.bad_rows)
                assert np.array_equal(yp, yu), (name, label, "pairs", unroll)
                ref = sp.csr_matrix((v, ci, rp), shape=(len(rp) - 1, ncols)) @ x
                np.testing.assert_allclose(yu, ref, rtol=1e-14, atol=1e-14)
                assert np.array_equal(yu, y), (name, label, unroll)  # entry order kept: the plain layout's bits
        if L.group > 1 and not fg:
            # 8-byte values take SELL-64 from fewer rows on (choose_group): the same matrix one row per lane
            L1 = Layout(np.asarray(rp), np.asarray(ci), np.asarray(v), ncols, 1)
            y1, acc1 = replay_one_row_per_lane(L1, x)
            assert acc1.bad_loads == 0 and acc1.bad_gathers == 0, (name, label, "SELL-64", acc1.bad_loads,
                                                                  acc1.bad_gathers)
            np.testing.assert_allclose(y1, y, rtol=1e-13, atol=1e-13)
        if cf is None:  # every operator but the prolongations (whose unit-row layout comes first)
            D = DiaLayout(rp, ci, v, ncols)
            for vb in (4, 8):
                if not D.use(vb, L.group):
                    continue
                dia_used.add(label)
                ye, ae = replay_dia_exact(D, x)
                assert ae.clean(), (name, label, "slice-diagonal exact chunks, one row", ae.bad)
                assert np.array_equal(ye, y), (name, label, "exact")  # the plain layout's bits (up to the sign of 0)
                if vb == 4 and ncols == len(rp) - 1 and ncols >= 2:  # FP32 square: the two-rows-per-lane kernel
                    yp, ap = replay_dia_pairs(D, x)
                    assert ap.clean(), (name, label, "slice-diagonal, two rows per lane", ap.bad)
                    assert np.array_equal(yp, ye), (name, label, "two rows per lane")
                    pairs_used.add(label)
    # the natural-order stencils take the form on level 0 (A, its strict parts, its FP64 copy); a random
    # relabelling scatters the offsets and keeps SELL-64
    if name.startswith("permuted"):
        assert not any(lbl.startswith("A0") for lbl in dia_used), dia_used
    else:
        assert {"A0", "A0 fp64", "A0 lower", "A0 upper"} <= dia_used, dia_used
        assert {"A0 lower", "A0 upper"} <= pairs_used, pairs_used


def test_unit_layout_needs_its_masks():
    """The unit-row layout stores each F row's entries with the stride of its slice's F-row count, and a 16-bit
    offset relative to that row's own diagonal base. Read as plain SELL-64 (the masks not reaching the
    kernel), lanes decode other rows' offsets against their own base and gather outside e; with the masks
    every access stays in range."""
    A = config_system("c2", 24)[0]
    found = 0
    for label, rp, ci, v, ncols, fg, cf in hierarchy_operators(namg_module(), A):
        if cf is None:
            continue
        Lu = UnitLayout(np.asarray(rp), np.asarray(ci), np.asarray(v), ncols, cf)
        plain = Layout(np.asarray(rp), np.asarray(ci), np.asarray(v), ncols)
        plain.ptr, plain.idx, plain.val, plain.stored = Lu.ptr, Lu.idx, Lu.val, Lu.stored
        x = np.random.default_rng(1).standard_normal(ncols)
        _, wrong = replay_one_row_per_lane(plain, x)
        _, right = replay_prolong_unit_rows(Lu, x)
        _, pairs = replay_prolong_unit_pairs(Lu, x)
        found += wrong.bad_gathers
        assert right.bad_gathers == 0 and right.bad_loads == 0, label
        assert pairs.bad_gathers == 0 and pairs.bad_loads == 0 and pairs.bad_table == 0 and pairs.bad_rows == 0, label
    assert found > 0


def namg_module():
    import paper_2112_14681_amd as m

    return m
