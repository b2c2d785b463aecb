"""Lane-level CPU model of the LPT loop of the partition kernels (the narrow
form for at most 64 bins): one key per lane, single steps, rounds of equal
weights and prefix rounds, re-sorted by the same 64-lane bitonic network.
It must place every component exactly as sequential LPT does (Section 4.3:
components by decreasing weight, each to the least loaded bin, ties to the
lower bin index).  The GPU parity tests check the kernels themselves."""
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
