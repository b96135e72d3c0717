"""Pins for the FP64 oracle: checks against facts that do not come from the oracle itself.

Each ``pin_*`` function raises AssertionError on failure.  The sources of truth are
  * the paper's definitions of s+/-, dl+/- and Eq. 2 (Sec. II-B), evaluated literally
    (the printed 1/2 -+ 1/2 erf form) in mpmath with >= 500 significant digits, with derivatives by
    mpmath's high-precision numerical differentiation;
  * scipy.special.log_ndtr as an independent library for log Phi;
  * closed forms (delta = mu, two vertices, coincident points), identities
    (s+ + s- = 1, reflection, the Eq. 5 rearrangement), invariances (translation,
    rotation, torque, scale) and central finite differences of the oracle's own loss;
  * brute force in pure Python + mpmath on tiny graphs.
The same list runs against planted-mistake builds of the oracle in test_oracle_mutants.py.
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np
from scipy.special import log_ndtr

import oracle
from paper_2011_03479_amd import synth

MU, SIGMA = 1.5, 1.0


# ----------------------------------------------------------------------------------------
# literal evaluation of the paper's definitions (Sec. II-B) in high-precision arithmetic
# ----------------------------------------------------------------------------------------

def _digits(delta, mu, sigma):
    """Working digits so that 1/2 -+ 1/2 erf keeps >= 500 significant digits at delta."""
    t = (float(delta) - mu) / sigma
    return 500 + int(0.22 * t * t)


def mp_dl(delta, edge, mu=MU, sigma=SIGMA):
    """dl+/- exactly as printed: -log2(1/2 -+ 1/2 erf((delta - mu)/(sqrt2 sigma)))."""
    with mp.workdps(_digits(delta, mu, sigma)):
        z = (mp.mpf(delta) - mp.mpf(mu)) / (mp.sqrt(2) * mp.mpf(sigma))
        s = mp.mpf(1) / 2 - mp.erf(z) / 2 if edge else mp.mpf(1) / 2 + mp.erf(z) / 2
        return -mp.log(s, 2)


def mp_dl_derivs(delta, edge, mu=MU, sigma=SIGMA):
    """(dl, dl', dl'') with central differences of step 1e-150 at >= 500 digits."""
    with mp.workdps(_digits(delta, mu, sigma)):
        f = lambda x: mp_dl(x, edge, mu, sigma)  # noqa: E731
        x = mp.mpf(delta)
        h = mp.mpf(10) ** -150
        return f(x), mp.diff(f, x, 1, h=h), mp.diff(f, x, 2, h=h)


def close(a, b, rel=1e-12, abs_=1e-300):
    a = float(a)
    b = float(b)
    return abs(a - b) <= rel * abs(b) + abs_


# ----------------------------------------------------------------------------------------
# pins on the pair function
# ----------------------------------------------------------------------------------------

PAIR_GRID = [0.0, 0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.5, 6.0, 10.0, 20.0, 30.0, 36.4, 36.6, 40.0, 60.0]
PARAMS = [(1.5, 1.0), (2.0, 0.5), (0.7, 1.7)]


def pin_pair_vs_mpmath():
    for mu, sigma in PARAMS:
        for delta in PAIR_GRID:
            if abs(delta - mu) / sigma > 60.0:
                continue
            for edge in (True, False):
                dl, d1, d2 = oracle.pair(delta, edge, mu, sigma)
                rdl, rd1, rd2 = mp_dl_derivs(delta, edge, mu, sigma)
                assert close(dl, rdl, 1e-12), (mu, sigma, delta, edge, dl, rdl)
                assert close(d1, rd1, 1e-10), (mu, sigma, delta, edge, d1, rd1)
                assert close(d2, rd2, 1e-8), (mu, sigma, delta, edge, d2, rd2)


def pin_pair_vs_scipy():
    """-log2 Phi(tau) against scipy's log_ndtr over edge and non-edge ranges."""
    for mu, sigma in PARAMS:
        for edge in (True, False):
            deltas = np.linspace(0.0, mu + 60 * sigma, 1201)
            for delta in deltas:
                a = -1.0 if edge else 1.0
                tau = a * (delta - mu) / sigma
                dl, d1, _ = oracle.pair(delta, edge, mu, sigma)
                ref = -log_ndtr(tau) / math.log(2)
                # a far tail is as exact as exp(-tau^2/2) of a rounded tau: ~tau^2 ulp
                rel = 1e-14 * (4.0 + tau * tau)
                assert close(dl, ref, rel, 1e-300), (edge, delta, dl, ref)
                # R = phi/Phi from the same library: d1 = -(a/sigma) R / ln2
                logR = -0.5 * tau * tau - 0.5 * math.log(2 * math.pi) - log_ndtr(tau)
                ref1 = -(a / sigma) * math.exp(logR) / math.log(2)
                assert close(d1, ref1, 4 * rel, 1e-300), (edge, delta, d1, ref1)


def pin_pair_closed_forms():
    # delta = mu: s+ = s- = 1/2, so dl = 1 bit; slope +-sqrt(2/pi)/(sigma ln 2)
    for mu, sigma in PARAMS:
        for edge in (True, False):
            dl, d1, _ = oracle.pair(mu, edge, mu, sigma)
            assert close(dl, 1.0, 1e-15)
            slope = math.sqrt(2 / math.pi) / (sigma * math.log(2))
            assert close(d1, slope if edge else -slope, 1e-14)
    # reflection: dl+(mu + D) = dl-(mu - D), d dl+(mu + D) = -d dl-(mu - D)
    for D in (0.3, 1.0, 1.5):
        a = oracle.pair(MU + D, True)
        b = oracle.pair(MU - D, False)
        assert close(a[0], b[0], 1e-14) and close(a[1], -b[1], 1e-13)
    # s+ + s- = 1 (the two probabilities of Sec. II-B are complementary)
    for delta in (0.0, 0.7, 1.5, 2.9, 5.0):
        p = 2.0 ** -oracle.pair(delta, True)[0] + 2.0 ** -oracle.pair(delta, False)[0]
        assert close(p, 1.0, 1e-14)


# ----------------------------------------------------------------------------------------
# pins on the whole-graph loss / gradient
# ----------------------------------------------------------------------------------------

def _graph_from_edges(n, edges):
    u = np.array([e[0] for e in edges], dtype=np.int64)
    v = np.array([e[1] for e in edges], dtype=np.int64)
    return synth.csr_from_edges(n, u, v)


def pin_two_vertices():
    X = np.array([[0.0, 0.0], [3.0, 4.0]])
    for edge in (True, False):
        g = _graph_from_edges(2, [(0, 1)] if edge else [])
        r = oracle.loss_grad(X, g.row_ptr, g.col_idx)
        dl, d1, _ = mp_dl_derivs(5.0, edge)
        assert close(r["loss"], dl, 1e-13)
        g1 = float(d1) * (X[0] - X[1]) / 5.0
        assert np.allclose(r["grad"][0], g1, rtol=1e-10, atol=0)
        assert np.allclose(r["grad"][1], -g1, rtol=1e-10, atol=0)
        assert r["edge_hits"] == (1 if edge else 0)


def pin_coincident_points():
    g = synth.erdos_renyi(9, 3.0, seed=11)
    X = np.full((9, 3), 0.37)
    r = oracle.loss_grad(X, g.row_ptr, g.col_idx)
    N = 9 * 8 // 2
    ref = g.m * float(mp_dl(0.0, True)) + (N - g.m) * float(mp_dl(0.0, False))
    assert close(r["loss"], ref, 1e-13)
    assert np.all(r["grad"] == 0.0)
    assert r["edge_hits"] == g.m


def pin_brute_force_tiny():
    """Pure Python + mpmath over all pairs of a 6-vertex graph (loss, gradient, hits)."""
    rng = np.random.default_rng(5)
    n, d = 6, 2
    X = rng.standard_normal((n, d))
    edges = [(0, 1), (1, 2), (2, 5), (3, 4), (0, 5)]
    g = _graph_from_edges(n, edges)
    E = set(edges) | {(b, a) for a, b in edges}
    loss = mp.mpf(0)
    grad = [[mp.mpf(0)] * d for _ in range(n)]
    hits = 0
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            diff = [mp.mpf(float(X[i, k])) - mp.mpf(float(X[j, k])) for k in range(d)]
            delta = mp.sqrt(sum(t * t for t in diff))
            dl, d1, _ = mp_dl_derivs(delta, (i, j) in E)
            if i < j:
                loss += dl
                hits += (i, j) in E
            for k in range(d):
                grad[i][k] += d1 * diff[k] / delta
    r = oracle.loss_grad(X, g.row_ptr, g.col_idx)
    assert close(r["loss"], loss, 1e-13)
    assert np.allclose(r["grad"], np.array([[float(v) for v in row] for row in grad]),
                       rtol=1e-10, atol=1e-14)
    assert r["edge_hits"] == hits == len(edges)


def pin_finite_differences():
    for n, d, seed in ((8, 1, 1), (12, 2, 2), (10, 3, 3), (9, 8, 4)):
        g = synth.erdos_renyi(n, 0.35 * (n - 1), seed=seed)
        rng = np.random.default_rng(100 + seed)
        X = rng.standard_normal((n, d)) * 1.3
        G = oracle.loss_grad(X, g.row_ptr, g.col_idx)["grad"]
        h = 1e-6
        for i in range(n):
            for k in range(d):
                Xp = X.copy()
                Xm = X.copy()
                Xp[i, k] += h
                Xm[i, k] -= h
                fd = (oracle.loss_grad(Xp, g.row_ptr, g.col_idx, want_grad=False)["loss"]
                      - oracle.loss_grad(Xm, g.row_ptr, g.col_idx, want_grad=False)["loss"]) / (2 * h)
                assert abs(fd - G[i, k]) <= 1e-6 * max(1.0, abs(G[i, k])), (n, d, i, k, fd, G[i, k])


def pin_invariances():
    rng = np.random.default_rng(21)
    n, d = 40, 3
    g = synth.erdos_renyi(n, 5.0, seed=21)
    X = rng.standard_normal((n, d))
    r = oracle.loss_grad(X, g.row_ptr, g.col_idx)
    G = r["grad"]
    scale = np.abs(G).sum()
    # translation: the loss only sees differences, so the gradients sum to zero
    assert np.all(np.abs(G.sum(axis=0)) <= 1e-12 * scale)
    rt = oracle.loss_grad(X + np.array([3.0, -2.0, 0.5]), g.row_ptr, g.col_idx)
    assert close(rt["loss"], r["loss"], 1e-12)
    # rotation: DL(XQ) = DL(X), G(XQ) = G(X) Q
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    rq = oracle.loss_grad(X @ Q, g.row_ptr, g.col_idx)
    assert close(rq["loss"], r["loss"], 1e-12)
    assert np.allclose(rq["grad"], G @ Q, rtol=0, atol=1e-11 * np.abs(G).max())
    # no torque: sum_i x_i g_i^T is symmetric
    T = X.T @ G
    assert np.allclose(T, T.T, rtol=0, atol=1e-11 * np.abs(T).max())
    # scale covariance: DL(cX; c mu, c sigma) = DL(X; mu, sigma), G scales by 1/c
    c = 2.5
    rs = oracle.loss_grad(c * X, g.row_ptr, g.col_idx, mu=c * MU, sigma=c * SIGMA)
    assert close(rs["loss"], r["loss"], 1e-12)
    assert np.allclose(rs["grad"], G / c, rtol=0, atol=1e-12 * np.abs(G).max())


def pin_edge_hits_and_rows():
    g = synth.chung_lu(300, 8.0, 2.5, seed=7)
    X = synth.init_embedding(300, 2, 1007)
    r = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_row_loss=True)
    assert r["edge_hits"] == g.m
    # the row losses count every pair twice, the loss once
    assert close(r["row_loss"].sum(), 2 * r["loss"], 1e-12)
    sub = np.array([0, 17, 299, 123])
    rr = oracle.rows(X, g.row_ptr, g.col_idx, sub)
    assert np.allclose(rr["grad"], r["grad"][sub], rtol=1e-13, atol=0)
    assert np.allclose(rr["row_loss"], r["row_loss"][sub], rtol=1e-13, atol=0)
    assert int(np.sum(np.diff(g.row_ptr)[sub])) >= int(rr["upper_hits"].sum())


def pin_wm_parabola_two_vertices():
    """The parabola of Sec. II-C (Eqs. 3-4) touches dl with the same slope and curvature at the
    current distance.  On a two-vertex graph the oracle's z_0 is the pair's weight w and its
    y_0 (Eq. 5) is w (x_1 + s (x_0 - x_1)); with x_0 = 0 and x_1 = (delta, 0) this gives
    y_0 = w (delta - d).  The parabola p(t) = w (t - d)^2 + c has p' = 2 w (t - d) and p'' = 2 w,
    so 2 y_0 must equal dl'(delta) and 2 z_0 must equal dl''(delta), both taken here from the
    printed definition by high-precision differentiation.  A_0 is |dl'(delta)|."""
    for mu, sigma in ((1.5, 1.0), (0.7, 1.7)):
        for delta in (0.3, 1.0, 1.5, 2.2, 3.5, 6.0):
            for edge in (True, False):
                g = _graph_from_edges(2, [(0, 1)] if edge else [])
                X = np.array([[0.0, 0.0], [delta, 0.0]])
                r = oracle.rows(X, g.row_ptr, g.col_idx, np.array([0]), mu, sigma, wm=True)
                _, rd1, rd2 = mp_dl_derivs(delta, edge, mu, sigma)
                z0, y0 = float(r["z"][0]), r["y"][0]
                assert close(2.0 * z0, rd2, 1e-8), (mu, sigma, delta, edge, 2 * z0, rd2)
                assert close(2.0 * y0[0], rd1, 1e-8), (mu, sigma, delta, edge, 2 * y0[0], rd1)
                assert abs(y0[1]) <= 1e-300
                assert close(r["abs_slope"][0], abs(rd1), 1e-10), (delta, edge, r["abs_slope"][0], rd1)


def pin_wm_brute_force_tiny():
    """z_i, y_i (Eq. 5) and A_i = sum_j |dl'| on a 7-vertex graph against a pure-Python
    brute force over all pairs with mpmath derivatives of the printed definition: each
    pair's parabola weight is fixed by p'' = 2 w = dl'' and its target distance by
    p'(delta) = 2 w (delta - d) = dl' (Sec. II-C, Eqs. 3-4)."""
    rng = np.random.default_rng(8)
    n, d = 7, 3
    X = 0.8 * rng.standard_normal((n, d))
    edges = [(0, 1), (1, 2), (2, 6), (3, 4), (0, 6), (4, 5)]
    g = _graph_from_edges(n, edges)
    E = set(edges) | {(b, a) for a, b in edges}
    z = [mp.mpf(0)] * n
    A = [mp.mpf(0)] * n
    y = [[mp.mpf(0)] * d for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            xi = [mp.mpf(float(X[i, k])) for k in range(d)]
            xj = [mp.mpf(float(X[j, k])) for k in range(d)]
            delta = mp.sqrt(sum((a - b) ** 2 for a, b in zip(xi, xj)))
            _, d1, d2 = mp_dl_derivs(delta, (i, j) in E)
            w = d2 / 2
            target = delta - d1 / (2 * w)
            s = target / delta
            z[i] += w
            A[i] += abs(d1)
            for k in range(d):
                y[i][k] += w * (xj[k] + s * (xi[k] - xj[k]))
    r = oracle.rows(X, g.row_ptr, g.col_idx, np.arange(n), wm=True)
    for i in range(n):
        assert close(r["z"][i], z[i], 1e-9), (i, r["z"][i], z[i])
        assert close(r["abs_slope"][i], A[i], 1e-10), (i, r["abs_slope"][i], A[i])
        yref = np.array([float(v) for v in y[i]])
        assert np.allclose(r["y"][i], yref, rtol=1e-9, atol=1e-12 * float(z[i])), (i, r["y"][i], yref)


def pin_wm_identity():
    """Eq. 5 with derivative-matched parabolas equals x_i - g_i / (2 z_i), z_i > 0."""
    rng = np.random.default_rng(31)
    n, d = 25, 2
    g = synth.erdos_renyi(n, 4.0, seed=31)
    X = rng.standard_normal((n, d))
    Xn, r = oracle.wm_update(X, g.row_ptr, g.col_idx)
    G = oracle.loss_grad(X, g.row_ptr, g.col_idx)["grad"]
    assert np.all(r["z"] > 0)
    assert np.allclose(Xn, X - G / (2 * r["z"][:, None]), rtol=0, atol=1e-12)
    # the parabola weight is half the second derivative (checked at the pair level)
    for delta in (0.4, 1.5, 3.0):
        for edge in (True, False):
            _, _, d2 = oracle.pair(delta, edge)
            _, _, rd2 = mp_dl_derivs(delta, edge)
            assert close(d2, rd2, 1e-8)


# ----------------------------------------------------------------------------------------
# slope optimisation (Sec. III-F)
# ----------------------------------------------------------------------------------------

def _sigma_case():
    """Three blocks placed around three centres: edges are mostly short, non-edges long, so
    Eq. 2 has an interior minimum over sigma (for an unstructured embedding it decreases all
    the way to 1 bit per pair as sigma grows)."""
    g = synth.sbm(3, 20, 0.5, 0.02, seed=41, permute=False)
    rng = np.random.default_rng(42)
    centres = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 3.0]])
    X = centres[np.repeat(np.arange(3), 20)] + 0.6 * rng.standard_normal((60, 2))
    return g, X


def pin_histogram_counts():
    """Counts add up to N pairs and m edges; at d = 1 every pair's bin equals a brute force in
    numpy single precision (one rounding of the product, as the fused multiply-add gives)."""
    g = synth.erdos_renyi(50, 5.0, seed=43)
    X = synth.init_embedding(50, 1, seed=44)
    r2_max = float(4 * np.max((X - X[0]) ** 2) * 1.001)
    nb = 257
    ha, he = oracle.histogram(X, g.row_ptr, g.col_idx, nb, r2_max)
    assert int(ha.sum()) == 50 * 49 // 2 and int(he.sum()) == g.m
    inv_w = np.float32(nb / r2_max)
    bha = np.zeros(nb, np.int64)
    bhe = np.zeros(nb, np.int64)
    edges = {(int(i), int(j)) for i, j in g.edges_upper()}
    x = X[:, 0].astype(np.float32)
    for i in range(50):
        for j in range(i + 1, 50):
            df = np.float32(x[i] - x[j])
            r2 = np.float32(df * df)
            b = int(min(np.float32(r2 * inv_w), np.float32(nb - 1)))
            bha[b] += 1
            if (i, j) in edges:
                bhe[b] += 1
    assert np.array_equal(bha, ha.astype(np.int64)) and np.array_equal(bhe, he.astype(np.int64))
    X3 = synth.init_embedding(50, 3, seed=45)
    ha3, he3 = oracle.histogram(X3, g.row_ptr, g.col_idx, 64, float(4 * np.max(np.sum((X3 - X3[0]) ** 2, 1)) * 1.001))
    assert int(ha3.sum()) == 50 * 49 // 2 and int(he3.sum()) == g.m


def pin_sigma_minimises_loss():
    """The exact slope is a minimum of Eq. 2 over sigma (the pinned loss), with a vanishing
    central difference, and it scales with the embedding: sigma*(cX; c mu) = c sigma*(X; mu)."""
    g, X = _sigma_case()
    s = oracle.sigma_exact(X, g.row_ptr, g.col_idx, MU)
    assert 1e-2 < s < 1e2

    def DL(sig):
        return oracle.loss_grad(X, g.row_ptr, g.col_idx, MU, sig, want_grad=False)["loss"]

    base = DL(s)
    for f in (0.99, 0.999, 1.001, 1.01):
        assert DL(s * f) > base
    h = 1e-4
    slope_scale = abs(DL(s * 1.1) - DL(s * 0.9)) / (0.2 * s)
    assert abs(DL(s * (1 + h)) - DL(s * (1 - h))) / (2 * h * s) <= 1e-4 * max(slope_scale, 1.0)
    s3 = oracle.sigma_exact(3.0 * X, g.row_ptr, g.col_idx, 3.0 * MU)
    assert abs(s3 / s - 3.0) <= 1e-9


def pin_sigma_histogram_converges():
    """The histogram bisection approaches the exact slope as the bins get finer."""
    g, X = _sigma_case()
    s = oracle.sigma_exact(X, g.row_ptr, g.col_idx, MU)
    r2_max = float(4 * np.max(np.sum((X - X[0]) ** 2, 1)) * 1.001)
    errs = []
    for nb in (256, 16384):
        ha, he = oracle.histogram(X, g.row_ptr, g.col_idx, nb, r2_max)
        errs.append(abs(oracle.sigma_from_histogram(ha, he, r2_max, MU) / s - 1))
    assert errs[1] < 2e-5 and errs[1] < errs[0]


# ----------------------------------------------------------------------------------------
# negative sampling (Sec. III-C)
# ----------------------------------------------------------------------------------------

def _lcg_draw(state, n):
    """One step of the paper's LCG and its float mapping, in numpy single precision."""
    state = (1103515245 * state + 1) & 0xFFFFFFFF
    f = np.array([0x3F800000 | (state & 0x7FFFFF)], dtype=np.uint32).view(np.float32)[0]
    u = np.float32(np.float32(f * np.float32(n)) - np.float32(n))
    return state, int(np.floor(u))


def _splitmix_hi(x):
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return (x ^ (x >> 31)) >> 32


def pin_sampler():
    """Samples are non-neighbours drawn by the published LCG (replayed here in numpy), roughly
    uniform over the non-neighbours; with no non-edge the sample is dropped."""
    g = synth.erdos_renyi(120, 10.0, seed=51)
    seed = 987654321
    smp = oracle.sample_pairs(g.row_ptr, g.col_idx, g.n, seed, 32)
    nbr = [set(g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]].tolist()) for i in range(g.n)]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for e in range(g.nnz):
        i, j = int(rows[e]), int(g.col_idx[e])
        if i > j:
            assert smp[2 * e] == -1 and smp[2 * e + 1] == -1
            continue
        for side, v in ((0, i), (1, j)):
            c = int(smp[2 * e + side])
            assert 0 <= c < g.n and c != v and c not in nbr[v]
            # replay: first accepted draw of this sample's own generator
            st = _splitmix_hi(seed + 2 * e + side)
            for _ in range(32):
                st, cand = _lcg_draw(st, g.n)
                if 0 <= cand < g.n and cand != v and cand not in nbr[v]:
                    break
            assert cand == c
    # uniformity: many samples of one vertex's partner spread over its non-neighbours
    star = synth.csr_from_edges(40, np.zeros(5, np.int64), np.arange(1, 6, dtype=np.int64))
    counts = np.zeros(40)
    for sd in range(400):
        ss = oracle.sample_pairs(star.row_ptr, star.col_idx, 40, 1000 + sd, 32)
        counts[ss[0::2][ss[0::2] >= 0]] += 1   # partners of vertex 0 (the hub)
    allowed = np.arange(6, 40)
    assert counts[:6].sum() == 0
    expect = counts.sum() / allowed.size
    assert np.max(np.abs(counts[allowed] - expect)) < 5 * np.sqrt(expect) + 5
    k = 8
    iu, ju = np.triu_indices(k, 1)
    kg = synth.csr_from_edges(k, iu.astype(np.int64), ju.astype(np.int64))
    assert np.all(oracle.sample_pairs(kg.row_ptr, kg.col_idx, k, 3, 16) == -1)


def pin_sampled_step():
    """The sampled step is Eq. 5 over the multiset {edges} + {sampled pairs}, written out here
    with each pair's parabola fixed by the derivatives of the printed definition (mpmath);
    its loss is the dl summed over those pairs."""
    g = synth.erdos_renyi(30, 4.0, seed=61)
    X = np.random.default_rng(62).standard_normal((30, 2))
    Xn, loss, smp = oracle.sampled_step(X, g.row_ptr, g.col_idx, 77, 32)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    pairs = []
    for e in range(g.nnz):
        i, j = int(rows[e]), int(g.col_idx[e])
        if i < j:
            pairs.append((i, j, True))
            if smp[2 * e] >= 0:
                pairs.append((i, int(smp[2 * e]), False))
            if smp[2 * e + 1] >= 0:
                pairs.append((j, int(smp[2 * e + 1]), False))
    Y = np.zeros_like(X)
    Z = np.zeros(g.n)
    L = 0.0
    for a, b, edge in pairs:
        delta = float(np.linalg.norm(X[a] - X[b]))
        dl, d1, d2 = (float(v) for v in mp_dl_derivs(delta, edge))
        w = d2 / 2                              # p'' = 2 w = dl''   (Eqs. 3-4)
        s_ab = (delta - d1 / (2 * w)) / delta   # p'(delta) = 2 w (delta - d) = dl'
        Y[a] += w * (X[b] + s_ab * (X[a] - X[b]))
        Y[b] += w * (X[a] + s_ab * (X[b] - X[a]))
        Z[a] += w
        Z[b] += w
        L += dl
    ref = np.where(Z[:, None] > 0, Y / np.where(Z > 0, Z, 1)[:, None], X)
    assert np.allclose(Xn, ref, rtol=1e-12, atol=1e-12)
    assert close(loss, L, 1e-12)


def pin_shard_partition():
    """The shard split of the pair sum: the shards partition the pairs (their losses, gradients
    and edge hits add up to the whole; one shard is the whole), and shard s holds exactly the
    pairs whose smaller vertex lies in strip s or S-1-s when every shard has one strip pair
    (checked against the per-row upper-triangle losses of the row oracle)."""
    n, T = 150, 16
    g = synth.chung_lu(n, 6.0, 2.5, seed=3)
    X = synth.init_embedding(n, 3, seed=4)
    full = oracle.loss_grad(X, g.row_ptr, g.col_idx)
    scale = float(np.abs(full["grad"]).max())
    one = oracle.loss_grad_shard(X, g.row_ptr, g.col_idx, T, 1, 0)
    assert close(one["loss"], full["loss"], 1e-14) and one["edge_hits"] == full["edge_hits"]
    assert np.allclose(one["grad"], full["grad"], rtol=0, atol=1e-12 * scale)
    for G in (2, 3, 5):
        parts = [oracle.loss_grad_shard(X, g.row_ptr, g.col_idx, T, G, s) for s in range(G)]
        assert close(sum(p["loss"] for p in parts), full["loss"], 1e-12)
        assert sum(p["edge_hits"] for p in parts) == full["edge_hits"]
        assert np.allclose(sum(p["grad"] for p in parts), full["grad"], rtol=0, atol=1e-12 * scale)
    sub = np.array([0, 15, 16, 77, 149])
    part = oracle.loss_grad_shard(X, g.row_ptr, g.col_idx, T, 3, 1)
    assert np.allclose(oracle.rows_shard(X, g.row_ptr, g.col_idx, sub, T, 3, 1), part["grad"][sub], rtol=1e-13,
                       atol=1e-14 * scale)
    S = (n + T - 1) // T                                  # 10 strips: 5 strip pairs
    upper = oracle.rows(X, g.row_ptr, g.col_idx, np.arange(n))["upper_loss"]
    strip = np.array([upper[q * T:(q + 1) * T].sum() for q in range(S)])
    for s in range(S // 2):
        part = oracle.loss_grad_shard(X, g.row_ptr, g.col_idx, T, S // 2, s)
        assert close(part["loss"], strip[s] + strip[S - 1 - s], 1e-12), s


# the slowest pin last: the mutant test stops at the first pin that rejects a mutant
ALL_PINS = [
    pin_pair_vs_scipy,
    pin_pair_closed_forms,
    pin_two_vertices,
    pin_coincident_points,
    pin_brute_force_tiny,
    pin_finite_differences,
    pin_invariances,
    pin_edge_hits_and_rows,
    pin_wm_identity,
    pin_wm_parabola_two_vertices,
    pin_wm_brute_force_tiny,
    pin_histogram_counts,
    pin_sigma_minimises_loss,
    pin_sigma_histogram_converges,
    pin_sampler,
    pin_sampled_step,
    pin_shard_partition,
    pin_pair_vs_mpmath,
]
