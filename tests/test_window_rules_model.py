"""CPU models of the pruning rules inside the lane-per-pair DP kernels,
checked against the plain DP on cost matrices with a planted cheap path.

The kernels drop cells whose value exceeds the threshold tau (Sec. 4.2:
sparse DK keeps only cells <= tau; for DTW a path through such a cell ends
above tau as well).  Two rules decide which cells they never compute:

* the sparse-DK tube: a window of W rows, several columns per iteration
  over the same rows, that moves up past dead leading slots; a live top slot hands the pair over to
  the general DP, also in the last columns when the end row lies above the
  window;
* the banded DP's dead-group skipping: groups of G slots whose
  predecessors all exceed tau are skipped, NC columns per sweep.

Each model follows its kernel's rules step by step on one pair (a wave
with one live lane skips the most); the result must equal the plain DP's
value when that is <= tau and +inf otherwise, or be a hand-over."""
import numpy as np
import pytest

INF = np.float32(np.inf)
f32 = np.float32


def combine(dist, c, p):
    return max(c, p) if dist == "dk" else f32(c + p)


def plain_dp(C, dist, w=None):
    m, n = C.shape
    D = np.full((m, n), INF, np.float32)
    for i in range(m):
        for j in range(n):
            if w is not None and abs(i - j) > w:
                continue
            p = f32(0) if i == 0 and j == 0 else min(
                D[i - 1, j] if i else INF, D[i, j - 1] if j else INF,
                D[i - 1, j - 1] if i and j else INF)
            D[i, j] = combine(dist, C[i, j], p)
    return D[m - 1, n - 1]


def planted(rng, m, n, w=None):
    """Costs in [0.5, 3) with a monotone path of costs in [0, 0.3) (inside
    the band |i - j| <= w when one is given), sometimes a cheap row too."""
    C = rng.uniform(0.5, 3, (m, n)).astype(np.float32)
    i = j = 0
    C[0, 0] = rng.uniform(0, 0.3)
    while (i, j) != (m - 1, n - 1):
        mv = int(rng.integers(0, 3))
        if i == m - 1:
            mv = 1
        if j == n - 1:
            mv = 0
        if w is not None and mv == 0 and i + 1 - j > w:
            mv = 2
        if w is not None and mv == 1 and j + 1 - i > w:
            mv = 2
        i, j = (i + 1, j) if mv == 0 else (i, j + 1) if mv == 1 else (i + 1, j + 1)
        C[i, j] = rng.uniform(0, 0.3)
    if rng.random() < 0.3:
        C[int(rng.integers(0, m)), :] = rng.uniform(0, 0.4, n)
    return C


def tube(C, tau, W, NT=4):
    """Sparse DK in a moving W-row window, NT columns per iteration over
    the same rows: ('done', value) or ('fallback',)."""
    m, n = C.shape
    SH = min(2 * NT - 1, W - 1)
    Dv = [INF] * W
    lo = j = 0
    while True:
        def cost(r, c):
            return C[r, c] if r < m else INF
        V = [[INF] * W for _ in range(NT)]
        down, dgp = [INF] * NT, [INF] * NT
        diag0 = f32(0) if j == 0 else INF
        for k in range(W):
            prev = None
            for r in range(NT):
                cst = cost(lo + k, min(j + r, n - 1))
                if r == 0:
                    old = Dv[k]
                    v = max(cst, min(down[0], old, diag0))
                    diag0 = old
                else:
                    v = max(cst, min(down[r], prev, dgp[r]))
                    dgp[r] = prev
                down[r] = V[r][k] = prev = v
        slot = m - 1 - lo
        if j + NT - 1 >= n - 1:
            rend = n - 1 - j
            if slot >= W and any(V[r][W - 1] <= tau for r in range(rend + 1)):
                return ("fallback",)
            res = V[rend][slot] if 0 <= slot < W else INF
            return ("done", res if res <= tau else INF)
        if any(V[r][W - 1] <= tau for r in range(NT)):
            return ("fallback",)
        if not min(V[NT - 1]) <= tau:
            return ("done", INF)
        sh = 0
        while sh < SH and not V[NT - 1][sh] <= tau:
            sh += 1
        Dv = V[NT - 1][sh:] + [INF] * sh
        lo += sh
        j += NT


def band(C, w, W, G, NC, tau, dist):
    """Banded DP over slots (slot k of column c is row c - w + k) with
    dead-group skipping, NC columns per sweep, single columns at the end."""
    m = C.shape[0]
    wact = 2 * w + 1

    def cost(k, col):
        row = col - w + k
        return C[row, col] if k < wact and 0 <= row < m and col < m else INF

    Dv = [f32(0) if k == w else INF for k in range(W)]
    KS = W + NC - 1
    NG = (KS + G - 1) // G
    comp_prev = (1 << NG) - 1
    gs, g_last = max(0, w // G - 1), min(NG - 1, w // G)
    j = 0
    while j + NC - 1 < m:
        prv, cur = [INF] * NC, [INF] * NC
        gw, gl, glo = NG, -1, NG
        run = gs < NG
        comp_now = 0
        lmin_all = INF
        for g in range(NG):
            if g < gs or not run:
                if (comp_prev >> g) & 1:
                    for u in range(G):
                        sl = g * G + u - (NC - 1)
                        if g * G + u < KS and 0 <= sl < W:
                            Dv[sl] = INF
                continue
            comp_now |= 1 << g
            wmin = lmin = INF
            for u in range(G):
                k = g * G + u
                if k >= KS:
                    continue
                for r in range(NC):
                    sl = k - r
                    if not 0 <= sl < W:
                        cur[r] = INF
                        continue
                    if r == 0:
                        diag, left = Dv[sl], (Dv[sl + 1] if sl + 1 < W else INF)
                    else:
                        diag, left = prv[r - 1], cur[r - 1]
                    v = combine(dist, cost(sl, j + r), min(prv[r], diag, left))
                    cur[r] = v
                    if r == NC - 1:
                        Dv[sl] = v
                        wmin = min(wmin, v)
                        if sl <= g * G:
                            lmin = min(lmin, v)
                prv = list(cur)
            lmin_all = min(lmin_all, wmin)
            if wmin <= tau:
                if gw == NG:
                    gw, glo = g, (g - 1 if lmin <= tau else g)
                gl = g
            if g >= g_last:
                run = min(prv) <= tau
        comp_prev = comp_now
        gs, g_last = (max(0, glo) if gw < NG else NG), gl
        if (j + NC) // 8 != j // 8 and not lmin_all <= tau:
            return INF
        j += NC
    while j < m:
        down = INF
        for k in range(W):
            left = Dv[k + 1] if k + 1 < W else INF
            v = combine(dist, cost(k, j), min(down, Dv[k], left))
            Dv[k], down = v, v
        j += 1
    return Dv[w] if Dv[w] <= tau else INF


@pytest.mark.parametrize("NT", [2, 4])
def test_tube_window_rules_exact(NT):
    rng = np.random.default_rng(7 + NT)
    handed = 0
    for _ in range(3000):
        m, n = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        W = int(rng.choice([8, 16]))
        C = planted(rng, m, n)
        tau = f32(rng.choice([0.3, 0.5, 0.7, 1.0, 1.5, np.inf]))
        ex = plain_dp(C, "dk")
        r = tube(C, tau, W, NT)
        if r[0] == "fallback":
            handed += 1
            continue
        assert r[1] == (ex if ex <= tau else INF), (m, n, W, tau, ex, r)
    assert 0 < handed < 3000


def test_tube_end_row_above_window_is_handed_over():
    """Row 0 stays cheap up to the last column, which is cheap all the way
    up: the end row (39) is above any window that stayed at rows 0 .. W-1."""
    q = np.full(40, 1.5, np.float32)
    q[0] = 0
    t = np.zeros(40, np.float32)
    t[-1] = 0.75
    C = (q[:, None] - t[None, :]) ** 2
    assert plain_dp(C, "dk") == f32(0.5625)
    for W in (8, 16, 32):
        assert tube(C, f32(0.5625), W) == ("fallback",)


@pytest.mark.parametrize("dist", ["dtw", "dk"])
def test_band_dead_group_skipping_exact(dist):
    rng = np.random.default_rng(11 if dist == "dtw" else 12)
    for _ in range(1500):
        m, w = int(rng.integers(1, 40)), int(rng.integers(0, 12))
        G, NC = int(rng.choice([4, 8])), int(rng.choice([1, 2]))
        W = (2 * w + G) // G * G + G * int(rng.integers(0, 2))
        C = planted(rng, m, m, w)
        ex = plain_dp(C, dist, w)
        scale = ex if np.isfinite(ex) else f32(1)
        tau = f32(rng.choice([0.5, 0.9, 1.0, 1.1, 2.0]) * scale)
        if rng.random() < 0.2:
            tau = ex
        if rng.random() < 0.1:
            tau = INF
        got = band(C, w, W, G, NC, tau, dist)
        assert got == (ex if ex <= tau else INF), (m, w, W, G, NC, tau, ex, got)
