"""Host-side emulation of the index arithmetic of one work tile of the
generate-and-reduce kernel (main_tile in scs_kernels.hip): every LDS,
trigonometric-table, basis-table and global offset that a tile can form,
checked against the sizes of the buffers it addresses, over the 2^20-bin
two-channel layout the step benchmark uses (512-bin LDS blocks, 2048-bin
chunks, 256 particle slots per tile) and over adversarial supports and
edges: supports that start or end on chunk and block boundaries, one-bin
supports, runs of empty segments, edges on chunk boundaries, idle lanes and
the last particle of the buffer, with each lane's block level picked as the
tile picks it (the prologue's level, raised from the super-blocks where
longer blocks meet the same bounds; the mixed path's doubled lengths too).  The bin loop takes two bins per pass and
forms both bins' terms before either bin's events: the second bin of a pass
that has one bin left reads the next bin, at the block's end the spare bin
the LDS holds after the staged ones, and every table
index (the bin's phase, in 1/1024 cycles, masked to 10 bits and or-ed with
the zero-entry offset) lies in [0, 1024], the 1025 entries the table holds
(the zero entry included), whatever the phase; the same holds for the
variant that reads each bin's table entry one bin ahead.  Nothing here runs
on a GPU; it replays integer arithmetic."""
import numpy as np

K_TRIG = 1024
TAB_ENTRIES = K_TRIG + 1
K_REC = 8


def table_index(phase_units, tmask, toff):
    """The kernel's table index: the low 32 bits of (phase + 1.5 * 2^52) as an
    integer, masked with tmask and or-ed with toff."""
    t = np.asarray(phase_units, dtype=np.float64) + 1.5 * 2.0 ** 52
    bits = t.view(np.uint64) & np.uint64(0xFFFFFFFF)
    return (bits.astype(np.int64) & tmask) | toff


def emulate_tile(K, L, CB, N, NV, lanes_lg, lanes_klo, lanes_khi, bounds, P_total, slot0, chunk, n_chunks,
                 lg_levels, lanes_up=None, lg_max=11, mixed=False):
    """Replay the offsets of one tile (chunk, group of len(lanes) slots);
    bounds is the whole [P_total][N+1] edge array plus two spare entries, the
    lanes are particles slot0 .. slot0 + len - 1.  Returns the number of
    lane-bins visited.  Raises AssertionError at the first offset out of its
    buffer."""
    W = len(lanes_lg)
    if lanes_up is None:
        lanes_up = np.full((W, 2), INT32_MAX, dtype=np.int64)
    cbins = L * CB
    Kc = chunk * cbins
    Ke = min(Kc + cbins, K)
    n_bounds = P_total * (N + 1) + 2
    n_zs = P_total * N * 3
    n_rec = n_chunks * P_total * K_REC
    lds_doubles = (L + 1) * NV  # L staged bins and the spare one after them
    p = slot0 + np.arange(W)
    live = p < P_total
    lgb = np.where(live, lanes_lg, -1)
    lo = np.where(lgb >= 0, lanes_klo, 0)
    hi = np.where(lgb >= 0, lanes_khi, 0)
    lo = np.maximum(lo, Kc)
    hi = np.minimum(hi, Ke)
    has = lo < hi

    def lev(i, k):
        return level_at(lgb[i], lanes_up[i], k, lg_max, mixed)

    lg = np.array([lev(i, lo[i]) for i in range(W)])
    if not has.any():
        return 0
    prow = np.where(live, p, slot0) * (N + 1)

    def bo(idx):
        assert np.all((idx >= 0) & (idx < n_bounds)), "edge read out of the bounds buffer"
        return bounds[idx]

    lgw = int(lg[has].min())
    # segment state
    n = np.zeros(W, dtype=np.int64)
    nb = np.full(W, 2 ** 31 - 1, dtype=np.int64)
    nb2 = nb.copy()
    for i in np.flatnonzero(has):
        row = bounds[prow[i]:prow[i] + N]
        n[i] = np.searchsorted(row, lo[i], side="right") - 1  # largest n in [0, N-1] with b_n <= lo
        nb[i] = bo(prow[i] + n[i] + 1)
        nb2[i] = bo(prow[i] + n[i] + 2)
    before = np.array([has[i] and bounds[prow[i] + n[i]] < Kc for i in range(W)])
    nxt = np.where(has, np.where(lo > Kc, lo, nb), 2 ** 31 - 1)
    rec_base = ((chunk - 0) * P_total + np.where(live, p, 0)) * K_REC
    zsp = (np.where(live, p, slot0) * N + n) * 3
    dst_rec = before.copy()
    dst_zs = zsp.copy()

    def store(i):
        if dst_rec[i]:
            off = rec_base[i]
            assert 0 <= off and off + 2 < n_rec, "head-record store out of rec"
        else:
            off = dst_zs[i]
            assert 0 <= off and off + 2 < n_zs, "segment store out of zs"

    def handle(i, k):
        store(i)
        if nb[i] <= k:
            n[i] += 1
            zsp[i] += 3
            nb[i] = nb2[i] if n[i] < N else 2 ** 31 - 1
            nb2[i] = bo(prow[i] + n[i] + 2)
            if nb[i] <= k:
                row = bounds[prow[i]:prow[i] + N]
                n[i] = np.searchsorted(row, k, side="right") - 1
                nb[i] = bo(prow[i] + n[i] + 1)
                if nb[i] <= k:
                    n[i] = N
                    nb[i] = 2 ** 31 - 1
                nb2[i] = bo(prow[i] + n[i] + 2)
                zsp[i] = (np.where(live, p, slot0)[i] * N + n[i]) * 3
            dst_rec[i] = False
            dst_zs[i] = zsp[i]
        nxt[i] = nb[i]

    have = np.full(W, -1, dtype=np.int64)
    tmask = np.zeros(W, dtype=np.int64)
    toff = np.full(W, K_TRIG, dtype=np.int64)
    rng = np.random.default_rng(chunk)
    visited = 0
    for b0 in range(Kc, Ke, L):
        b1 = min(b0 + L, Ke)
        nbins = b1 - b0
        # the staged bins, then the zeroed spare bin after them
        assert b1 * NV <= K * NV and (nbins + 1) * NV <= lds_doubles, "staging out of the bin table or the LDS block"
        llo = np.maximum(lo, b0)
        lhi = np.minimum(hi, b1)
        act = llo < lhi
        if not act.any():
            continue
        wlo, whi = int(llo[act].min()), int(lhi[act].max())
        Lp = 1 << lgw
        for sb0 in range((wlo >> lgw) << lgw, whi, Lp):
            s_lo, s_hi = max(sb0, wlo), min(sb0 + Lp, whi)
            sact = act & (llo < sb0 + Lp) & (lhi > sb0)
            lgl = np.array([lev(i, sb0) if has[i] else lgw for i in range(W)])
            assert np.all(lgl[sact] >= lgw) and np.all(lgl <= lg_max), "a lane's level below the wave's step"
            sbl = (sb0 >> lgl) << lgl
            setup = sact & (have != sbl)
            for i in np.flatnonzero(setup):
                sub = sbl[i] >> lgl[i]
                assert 0 <= sub < lg_levels[lgl[i]], "basis-table entry out of its level"
                # the block lies inside one super-block, at one level throughout
                assert sbl[i] >> lg_max == (sbl[i] + (1 << lgl[i]) - 1) >> lg_max
                assert lev(i, sbl[i]) == lgl[i] == lev(i, sbl[i] + (1 << lgl[i]) - 1)
                have[i] = sbl[i]
                tmask[i], toff[i] = K_TRIG - 1, 0
            for k in range(s_lo, s_hi, 2):
                two = k + 1 < s_hi
                # both bins' data and table entries first: any phase (random,
                # huge, negative) gives a table index in range
                for kb in (k, k + 1):
                    off = (kb - b0) * NV
                    # a pass with one bin left reads the next bin, at most the
                    # spare one after the staged block
                    assert 0 <= off and off + NV <= (nbins + 1) * NV <= lds_doubles, "bin read out of the staged block"
                    ph = rng.uniform(-2.0 ** 40, 2.0 ** 40, size=(2, W))
                    for q in (table_index(ph[0], tmask, toff), table_index(ph[1], tmask, toff)):
                        assert np.all((q >= 0) & (q < TAB_ENTRIES)), "table index out of the table"
                # then each bin's events, before its terms enter the sums
                for kb in ((k, k + 1) if two else (k,)):
                    for i in np.flatnonzero(nxt <= kb):
                        handle(i, kb)
                    visited += W
    # chunk close: the open segment's sums
    for i in np.flatnonzero(has & (n < N)):
        if nb[i] <= hi[i]:
            store(i)
        else:
            off = rec_base[i] + (0 if dst_rec[i] else 3)
            assert off + 2 < n_rec
    return visited


NO_BIN = 2.0 ** 40
INT32_MAX = 2 ** 31 - 1


def super_ups(lgb, kup, lg_max):
    """The tile's thresholds for one lane (the kernel's rule): the first
    super-block start (a multiple of 2^lg_max) at or after each bin from which
    two and four times the prologue's block length meet the bounds, or
    INT32_MAX."""
    ups = [INT32_MAX, INT32_MAX]
    if 3 <= lgb < lg_max:
        sup = float(1 << lg_max)
        u = [np.ceil(kup[0] / sup) * sup, np.ceil(kup[1] / sup) * sup]
        ups[0] = int(u[0]) if u[0] < INT32_MAX else INT32_MAX
        ups[1] = int(u[1]) if (lgb + 2 <= lg_max and u[1] < INT32_MAX) else INT32_MAX
    return ups


def level_at(lgb, ups, k, lg_max, mixed=False):
    """The lane's block level at bin k (the kernel's rule)."""
    lev = lgb + (k >= ups[0]) + (k >= ups[1])
    if mixed and 0 <= lev < lg_max:
        lev += 1
    return int(lev)


def _edges(rng, klo, khi, N, kind):
    if kind == "equal":
        e = np.sort(rng.integers(klo, khi + 1, size=N - 1))
    elif kind == "runs":  # long runs of empty segments and one-bin segments
        e = np.sort(np.concatenate([np.full((N - 1) // 2, klo + (khi - klo) // 3),
                                    rng.integers(klo, khi + 1, size=N - 1 - (N - 1) // 2)]))
    else:  # edges on chunk and block boundaries
        grid = np.arange((klo // 512) * 512, khi + 1, 512)
        e = np.sort(np.clip(rng.choice(grid, size=N - 1), klo, khi))
    return np.concatenate([[klo], e, [khi]]).astype(np.int64)


def test_tile_offsets_stay_in_their_buffers():
    K, L, CB, NV = 1 << 20, 512, 4, 6
    N = 64
    W = 256
    P_total = 3 * W - 17  # a partial last group
    n_chunks = (K + L * CB - 1) // (L * CB)
    lg_levels = {lg: (K + (1 << lg) - 1) >> lg for lg in range(3, 12)}
    rng = np.random.default_rng(2408)
    lg = rng.integers(3, 12, size=P_total)
    klo = rng.integers(0, K, size=P_total)
    span = rng.choice([1, 2, 7, 500, 2048, 4096, 100000], size=P_total)
    khi = np.minimum(klo + span, K)
    # supports starting or ending exactly on chunk / block boundaries, the
    # band's edges, invalid and empty ones
    klo[:8] = [0, 2048, 2047, 512, K - 1, K - 2048, 4096, 0]
    khi[:8] = [2048, 4096, 2049, 1024, K, K, 4097, K]
    lg[8], khi[9] = -1, klo[9]
    # bins from which two and four times the prologue's length hold: inside
    # the support, at its start, or never
    u0 = klo + rng.integers(0, np.maximum(khi - klo, 1))
    u1 = u0 + rng.integers(0, np.maximum(khi - u0, 1))
    kup = np.stack([u0, u1], axis=1).astype(np.float64)
    kup[rng.random(P_total) < 0.25] = NO_BIN
    kup[rng.random(P_total) < 0.1, 1] = NO_BIN
    kup[10:14, 0] = klo[10:14]
    kinds = ["equal", "runs", "boundary"]
    bounds = np.concatenate([np.concatenate([_edges(rng, klo[i], khi[i], N, kinds[i % 3]) if khi[i] > klo[i]
                                             else np.full(N + 1, klo[i]) for i in range(P_total)]),
                             [0, 0]])
    chunks = sorted({0, 1, 2, n_chunks - 1, n_chunks - 2} | {int(c) for c in klo[:8] // (L * CB)} |
                    {int(c) for c in rng.integers(0, n_chunks, size=6)})
    total = 0
    for g0 in range(0, P_total, W):
        sl = slice(g0, min(g0 + W, P_total))
        pad = W - (sl.stop - sl.start)
        kl = np.concatenate([klo[sl], np.zeros(pad, dtype=np.int64)])
        kh = np.concatenate([khi[sl], np.zeros(pad, dtype=np.int64)])
        lgs = np.concatenate([lg[sl], np.full(pad, -1)])
        ups = np.array([super_ups(lg[i], kup[i], 11) for i in range(sl.start, sl.stop)] +
                       [[INT32_MAX, INT32_MAX]] * pad, dtype=np.int64)
        for c in chunks:
            for mixed in (False, True):
                total += emulate_tile(K, L, CB, N, NV, lgs, kl, kh, bounds, P_total, g0, c, n_chunks, lg_levels,
                                      ups, 11, mixed)
    print(f"lane-bins replayed: {total}")
    assert total > 0


def test_block_level_rule():
    """Every block of a raised level starts at or after the bin from which
    that level meets the bounds; the level never falls below the prologue's,
    never rises above lg_max, never falls as the bin rises, and changes only
    at super-block starts, so it does not depend on the chunk length."""
    rng = np.random.default_rng(13170)
    K, lg_max = 1 << 20, 11
    for _ in range(2000):
        lgb = int(rng.integers(3, lg_max + 1))
        u0 = float(rng.integers(0, K))
        u1 = u0 + float(rng.integers(0, K))
        kup = [np.array([u0, u1]), np.array([u0, NO_BIN]), np.array([NO_BIN, NO_BIN])][int(rng.integers(0, 3))]
        ups = super_ups(lgb, kup, lg_max)
        ks = np.sort(rng.integers(0, K, size=64))
        prev = -1
        for k in ks:
            k = int(k)
            lev = level_at(lgb, ups, k, lg_max)
            assert lgb <= lev <= lg_max and lev >= prev
            prev = lev
            first = (k >> lev) << lev  # the start of the block holding bin k
            for i in range(lev - lgb):
                assert first >= kup[i]
            s0 = (k >> lg_max) << lg_max
            assert level_at(lgb, ups, s0, lg_max) == lev == level_at(lgb, ups, s0 + (1 << lg_max) - 1, lg_max)
            mix = level_at(lgb, ups, k, lg_max, mixed=True)
            assert mix == min(lev + 1, lg_max)


def test_table_index_range_for_any_phase():
    """The masked index covers [0, 1023] for a lane with polynomials and is
    the zero entry 1024 before a lane's first block, for ordinary, huge,
    negative, infinite and NaN phases alike."""
    ph = np.concatenate([np.linspace(-5000, 5000, 10001), [0.0, -0.0, 2.0 ** 51, -2.0 ** 51, 1e300, -1e300,
                                                           np.inf, -np.inf, np.nan]])
    q = table_index(ph, K_TRIG - 1, 0)
    assert q.min() >= 0 and q.max() <= K_TRIG - 1
    assert np.all(table_index(ph, 0, K_TRIG) == K_TRIG)
    # for |phase| < 2^51 the entry is the nearest 1/1024 cycle, mod 1024
    mid = np.linspace(-3000.4, 3000.4, 77)
    assert np.array_equal(table_index(mid, K_TRIG - 1, 0), np.mod(np.rint(mid).astype(np.int64), K_TRIG))
