"""The one-pass merge of the column statistics as algebra, in float32 on the CPU: the
pairwise (count, mean, M2) combination (Chan, Golub and LeVeque) of per-segment partials,
beside a Neumaier-compensated total, gives the deviation the FP64 definition gives, on
inputs with large column offsets; a plain one-pass sum of squares does not."""
import numpy as np

from paper_1810_10496_amd import synth

F = np.float32


def neumaier(s, c, x):
    t = F(s + x)
    if abs(s) >= abs(x):
        c = F(c + F(F(s - t) + x))
    else:
        c = F(c + F(F(x - t) + s))
    return t, c


def combine(cnt, mu, m2, nb, mb, m2b):
    if nb <= 0:
        return cnt, mu, m2
    if cnt == 0:
        return F(nb), F(mb), F(m2b)
    t = F(cnt + nb)
    rt = F(F(1) / t)
    d = F(mb - mu)
    return t, F(mu + F(F(d * F(nb)) * rt)), F(m2 + F(m2b + F(F(d * d) * F(F(cnt * F(nb)) * rt))))


def merged_std(col, rows, waves=8):
    """Per-segment (compensated sum, M2 about the segment mean) rounded to float32, folded
    wavefront by wavefront (segments w, w+waves, ...) and the wavefronts in order."""
    n = len(col)
    part = []
    for r0 in range(0, n, rows):
        x = col[r0:r0 + rows].astype(np.float64)
        s = x.sum()
        hi = F(s)
        part.append((hi, F(s - float(hi)), F(((x - s / len(x)) ** 2).sum()), len(x)))
    acc = []
    for w in range(waves):
        h = lo = cnt = mu = m2 = F(0)
        for hv, lv, mv, nb in part[w::waves]:
            h, lo = neumaier(h, lo, hv)
            h, lo = neumaier(h, lo, lv)
            cnt, mu, m2 = combine(cnt, mu, m2, F(nb), F(F(hv + lv) / F(nb)), mv)
        acc.append((h, lo, cnt, mu, m2))
    th = tl = tc = tm = t2 = F(0)
    for h, lo, c, mu, m2 in acc:
        th, tl = neumaier(th, tl, h)
        th, tl = neumaier(th, tl, lo)
        tc, tm, t2 = combine(tc, tm, t2, c, mu, m2)
    return F((th + tl) / F(n)), np.sqrt(F(t2 / F(n - 1)))


def test_pairwise_merge_matches_the_fp64_deviation():
    for n, m, rows in ((2048, 16, 64), (1000, 12, 16), (130, 8, 16), (2, 4, 64)):
        X, _ = synth.corr_inputs(n, m)
        X = X.astype(np.float32)
        for j in range(m):
            col = X[:, j]
            ref = col.astype(np.float64)
            mu, sd = merged_std(col, rows)
            assert abs(float(mu) - ref.mean()) <= 1e-6 * np.abs(ref).mean()
            assert abs(float(sd) - ref.std(ddof=1)) <= 1e-6 * ref.std(ddof=1)


def test_offsets_defeat_a_naive_one_pass_but_not_the_merge():
    rng = np.random.default_rng(7)
    col = (1e4 + rng.standard_normal(4096)).astype(np.float32)
    ref = col.astype(np.float64).std(ddof=1)
    s = F(0)
    q = F(0)
    for x in col:
        s = F(s + x)
        q = F(q + F(x * x))
    naive = np.sqrt(max(F(F(q - F(s * s) / F(len(col))) / F(len(col) - 1)), F(0)))
    assert abs(float(naive) - ref) > 0.1 * ref
    # what is left is the float32 rounding of the segment means at 1e4 (about 4e-6 here;
    # the two-pass form, about the total mean, gives 2e-6 on the same column)
    assert abs(float(merged_std(col, 64)[1]) - ref) <= 1e-5 * ref
