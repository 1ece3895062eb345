"""Per-atom error bound of the mixed-precision force path (test helper).

The mixed path evaluates each pair's force factor in FP32: 1/r^2 by the
hardware reciprocal (1 ulp), r^-6 by two products, lj1 r^-6 - lj2 with both
coefficients rounded to FP32, and two more products; forces, energy and
virial are accumulated in FP64 from those factors, and displacements, r^2 and
the cutoff test stay FP64.  Counting every rounding of that chain (u = 2^-24)
bounds the error of one pair's force by 25 u (lj1 r^-14 + lj2 r^-8) r and of
one pair's energy by 25 u (lj3 r^-12 + lj4 r^-6), with lj1 = 48 eps s^12,
lj2 = 24 eps s^6, lj3 = 4 eps s^12, lj4 = 4 eps s^6.  Summing those over an
atom's partners inside the cutoff gives the bound used in the parity tests:
|dF_i|_inf <= 25 u S_i with S_i = sum_j (lj1 r^-14 + lj2 r^-8) r.
"""
import numpy as np

U32 = 2.0 ** -24
K_PAIR = 25.0


def _coef(eps, sigma, ti, tj):
    e = eps[ti, tj]
    s = sigma[ti, tj]
    s6 = s ** 6
    return 48.0 * e * s6 * s6, 24.0 * e * s6, 4.0 * e * s6 * s6, 4.0 * e * s6


def pair_abs_sums(x, types, box, eps, sigma, rc, rows, counts, offsets, idx):
    """S_i (force), P_i (energy) and Q_i (virial: the force term times r) sums
    over the partners of rows[k] listed in CSR (counts, offsets, idx) that lie
    inside the pair cutoff."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    t = np.zeros(n, dtype=np.int64) if types is None else np.asarray(types, dtype=np.int64)
    eps, sigma, rc = (np.atleast_2d(np.asarray(a, dtype=np.float64)) for a in (eps, sigma, rc))
    box = np.asarray(box, dtype=np.float64)
    rows = np.asarray(rows)
    owner = np.repeat(np.arange(len(rows)), counts)
    i = rows[owner]
    j = idx[:offsets[-1]] if len(idx) else idx
    d = x[i] - x[j]
    d -= box * np.round(d / box)
    r2 = (d * d).sum(axis=1)
    inside = r2 < rc[t[i], t[j]] ** 2
    r = np.sqrt(r2)
    lj1, lj2, lj3, lj4 = _coef(eps, sigma, t[i], t[j])
    f_abs = np.where(inside, (lj1 * r ** -14 + lj2 * r ** -8) * r, 0.0)
    e_abs = np.where(inside, lj3 * r ** -12 + lj4 * r ** -6, 0.0)
    S = np.bincount(owner, weights=f_abs, minlength=len(rows))
    P = np.bincount(owner, weights=e_abs, minlength=len(rows))
    Q = np.bincount(owner, weights=f_abs * r, minlength=len(rows))
    return S, P, Q


def check_mixed(f, ev, f_ref, ev_ref, x, types, box, eps, sigma, rc, csr, rows=None,
                normwise=2e-6):
    """Mixed forces (rows of f, in the order of `rows`, all atoms if None)
    within the per-atom bound 25 u S_i of the FP64 reference, and within
    `normwise` of max |F_ref| overall; energy and virial (if given, full-list
    sums: each pair counted from both ends) within 25 u of half the summed
    P_i and Q_i.  Returns the largest |dF_i|_inf / S_i seen."""
    n = np.asarray(x).shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    counts, offsets, idx = csr
    S, P, Q = pair_abs_sums(x, types, box, eps, sigma, rc, rows, counts, offsets, idx)
    df = np.abs(np.asarray(f) - np.asarray(f_ref)).max(axis=1)
    assert np.all(df <= K_PAIR * U32 * S + 1e-300), float(np.max(df / np.maximum(S, 1e-300)))
    scale = np.abs(f_ref).max()
    assert df.max() <= normwise * (scale if scale > 0 else 1.0), df.max() / scale
    if ev is not None:
        de = np.abs(np.asarray(ev) - np.asarray(ev_ref))
        assert de[0] <= K_PAIR * U32 * 0.5 * P.sum(), (de[0], P.sum())
        assert np.all(de[1:] <= K_PAIR * U32 * 0.5 * Q.sum()), (de[1:], Q.sum())
    return float(np.max(df / np.maximum(S, 1e-300)))
