"""Lane-level CPU model of the LPT loop of the partition kernels (the narrow
form for at most 64 bins): one key per lane, single steps, rounds of equal
weights and prefix rounds, re-sorted by the same 64-lane bitonic network.
It must place every component exactly as sequential LPT does (Section 4.3:
components by decreasing weight, each to the least loaded bin, ties to the
lower bin index).  Two more models: the first round of LPT over more than
64 bins built in one pass, and the radix sort of the 1024-thread partition
kernel.  The GPU parity tests check the kernels themselves."""
import numpy as np

W = 64     # lanes of a wave: the bins of one window
RMIN = 6   # kLptRoundMin: equal-weight rounds from this many items
GMIN = 8   # kLptPrefixMin: prefix rounds from this many items


def lpt_seq(ws, P):
    order = sorted(range(len(ws)), key=lambda i: (-ws[i], i))
    load = [0] * P
    out = [0] * len(ws)
    for i in order:
        b = min(range(P), key=lambda b: (load[b], b))
        out[i] = b
        load[b] += ws[i]
    return out, load
def bitonic64(x):
    x = list(x)
    k = 2
    while k <= 64:
        j = k // 2
        while j > 0:
            p = [x[l ^ j] for l in range(64)]
            y = []
            for l in range(64):
                keep_min = ((l & j) == 0) == ((l & k) == 0)
                mn, mx = min(x[l], p[l]), max(x[l], p[l])
                y.append(mn if keep_min else mx)
            x = y
            j //= 2
        k *= 2
    return x
stats = {"step": 0, "eq": 0, "gen": 0, "scanfail": 0}
def lpt_emu(ws, P):
    order = sorted(range(len(ws)), key=lambda i: (-ws[i], i))
    kb = 0
    while (1 << kb) < P: kb += 1
    bmask = (1 << kb) - 1
    assert sum(ws) + 1 < (1 << (32 - kb))
    Wn = min(P, W)
    assert P <= W  # single window model
    key = [l if l < Wn else 0xFFFFFFFF for l in range(W)]
    out = [0] * len(ws)
    nc = len(ws)
    M32 = 0xFFFFFFFF
    for base in range(0, nc, W):
        cnt = min(nc - base, W)
        item = [order[base + l] if l < cnt else None for l in range(W)]
        iw = [(M32 - ws[item[l]]) if l < cnt else 0 for l in range(W)]
        mine = [0] * W
        t = 0
        while t < cnt:
            wt = iw[t]; q = M32 - wt
            k0 = key[0]; nk = k0 + (q << kb)
            below = [key[l] < nk for l in range(W)]
            same = [l < cnt and iw[l] == wt for l in range(W)][t:] + [False] * t
            run = 0
            while run < W and same[run]: run += 1
            m = sum(below)
            c = min(run, m)
            cgen = 0
            if m >= GMIN and c < m:
                # prefix round candidate
                qs = [M32 - iw[(l + t) & 63] for l in range(W)]
                has = [l < cnt - t and l < Wn for l in range(W)]
                r = [(key[l] + (qs[l] << kb)) if has[l] else M32 for l in range(W)]
                assert all(x <= M32 for x in r)
                # inclusive prefix min by shifts, then exclusive by one shift
                pm = list(r)
                d = 1
                while d < 64:
                    pm = [min(pm[l], pm[l - d]) if l >= d else pm[l] for l in range(W)]
                    d *= 2
                ex = [pm[l - 1] if l >= 1 else M32 for l in range(W)]
                ok = [has[l] and key[l] < ex[l] for l in range(W)]
                while cgen < W and ok[cgen]: cgen += 1
                assert cgen >= c
                if cgen < GMIN:
                    stats["scanfail"] += 1
            if cgen >= GMIN:
                stats["gen"] += 1
                src = [key[(l - t) & 63] for l in range(W)]
                for l in range(W):
                    if t <= l < t + cgen: mine[l] = src[l] & bmask
                x = [r[l] if l < cgen else key[l] for l in range(W)]
                key = bitonic64(x)
                assert key == sorted(x)
                t += cgen
            elif c >= RMIN:
                stats["eq"] += 1
                src = [key[(l - t) & 63] for l in range(W)]
                for l in range(W):
                    if t <= l < t + c: mine[l] = src[l] & bmask
                x = [key[l] + (q << kb) if l < c else key[l] for l in range(W)]
                key = sorted(x)
                t += c
            else:
                stats["step"] += 1
                p = sum(below) - 1
                for l in range(W):
                    if l == t: mine[l] = k0 & bmask
                nxt = [key[l + 1] if l < 63 else key[63] for l in range(W)]
                key = [nxt[l] if l < p else (nk if l == p else key[l]) for l in range(W)]
                t += 1
        for l in range(cnt):
            out[item[l]] = mine[l]
    load = [0] * P
    for l in range(Wn):
        load[key[l] & bmask] = key[l] >> kb
    return out, load


def test_lane_model_matches_sequential_lpt():
    rng = np.random.default_rng(2)
    for trial in range(160):
        P = int(rng.choice([1, 2, 3, 7, 16, 33, 63, 64]))
        n = int(rng.integers(0, 300))
        kind = trial % 4
        if kind == 0:
            ws = rng.integers(1, 6, size=n)
        elif kind == 1:
            ws = rng.integers(1, 200, size=n)
        elif kind == 2:
            ws = np.concatenate([rng.integers(100, 1000, size=n // 4), rng.integers(1, 4, size=n - n // 4)])
        else:
            ws = 2 ** rng.integers(0, 12, size=n)
        ws = [int(w) for w in ws]
        assert lpt_emu(ws, P) == lpt_seq(ws, P), (trial, P, n)
    # every kind of step was taken
    assert stats["step"] and stats["eq"] and stats["gen"]


def first_round_list(ws_sorted, P):
    """The sorted (load, bin) list after the first P items, as the partition
    kernel builds it in one pass for more than 64 bins: item t goes to bin t,
    and bin t sits after the bins past its run of equal weights, in bin order
    within the run."""
    out = [None] * P
    for t in range(P):
        wt = ws_sorted[t]
        g0 = next(g for g in range(t + 1) if ws_sorted[g] == wt)
        end = next((g for g in range(t, P) if ws_sorted[g] < wt), P)
        out[(P - end) + (t - g0)] = (wt, t)
    return out


def test_first_round_in_one_pass_matches_lpt():
    rng = np.random.default_rng(3)
    for P in (65, 100, 1024):
        for kind in ("uniform", "ties", "ones", "heavy"):
            m = P + int(rng.integers(1, 2 * P))
            if kind == "uniform":
                w = rng.integers(1, 10**6, m)
            elif kind == "ties":
                w = rng.integers(1, 6, m)
            elif kind == "ones":
                w = np.ones(m, dtype=int)
            else:
                w = (rng.pareto(1.1, m) * 10 + 1).astype(int)
            ws = sorted(w.tolist(), reverse=True)
            # sequential LPT over the first P items
            load = [0] * P
            for t in range(P):
                b = min(range(P), key=lambda b: (load[b], b))
                assert b == t, (P, kind, t)
                load[b] += ws[t]
            assert first_round_list(ws, P) == sorted((load[b], b) for b in range(P)), (P, kind)


def radix_hi16_model(keys, passes, nw):
    """The radix sort of the 1024-thread partition kernel, lane by lane: each
    of nw waves ranks 64 keys per round by digit (the lanes holding the same
    digit found by eight ballots) against its running count per digit, one
    scan over (digit, wave) counts in digit-major order gives the starts."""
    n = len(keys)
    per_w = (-(-n // nw) + 63) // 64 * 64
    src = list(keys)
    for p in range(passes):
        s = 16 + 8 * p
        cnt = [[0] * 256 for _ in range(nw)]
        rank = {}
        for w in range(nw):
            for r in range(per_w // 64):
                idx = [w * per_w + r * 64 + l for l in range(64)]
                valid = [i < n for i in idx]
                d = [(src[i] >> s) & 255 if v else 0 for i, v in zip(idx, valid)]
                ball = lambda pred: sum(1 << l for l in range(64) if pred(l))
                peers0 = ball(lambda l: valid[l])
                peers = []
                for l in range(64):
                    pm = peers0
                    for b in range(8):
                        m = ball(lambda k: valid[k] and (d[k] >> b) & 1)
                        pm &= m if (d[l] >> b) & 1 else ~m
                    peers.append(pm)
                before = [cnt[w][d[l]] for l in range(64)]
                for l in range(64):
                    if valid[l]:
                        rank[idx[l]] = before[l] + bin(peers[l] & ((1 << l) - 1)).count("1")
                        if peers[l] & ((1 << l) - 1) == 0:
                            cnt[w][d[l]] = before[l] + bin(peers[l]).count("1")
        flat = [cnt[e % nw][e // nw] for e in range(256 * nw)]
        start, acc = [0] * len(flat), 0
        for e, c in enumerate(flat):
            start[e], acc = acc, acc + c
        dst = [None] * n
        for i in range(n):
            w = i // per_w
            t = start[((src[i] >> s) & 255) * nw + w] + rank[i]
            assert 0 <= t < n and dst[t] is None
            dst[t] = src[i]
        src = dst
    return src


def test_radix_sort_model_is_a_stable_sort():
    rng = np.random.default_rng(5)
    for n, nw in ((1, 4), (63, 4), (200, 4), (513, 16), (1500, 16)):
        for kind in ("small", "uniform", "equal"):
            hi = {"small": rng.integers(0, 40, n), "uniform": rng.integers(0, 65536, n),
                  "equal": np.full(n, 9)}[kind]
            keys = [int(h) << 16 | i for i, h in enumerate(hi)]
            passes = 1 if hi.max() < 256 else 2
            assert radix_hi16_model(keys, passes, nw) == sorted(keys), (n, nw, kind)
