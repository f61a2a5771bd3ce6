"""The splitting schemes of the split-precision forms, checked on the CPU.

A plain NumPy model of the two slicings (written from their definitions, not
shared with the HIP code) pins the facts the GPU kernels rely on:

* every slice is an integer inside its stated range, so FP16 (|x| <= 2048)
  and int8 (|x| <= 127) hold it exactly;
* the slices reconstruct the scaled value up to the stated remainder;
* over one flush interval the leading levels of the FP16 form and every
  level of the INT8 form stay inside the exact range of their accumulator
  (2^24 for FP32, 2^31 for INT32), for worst-case (extreme) inputs;
* the truncated level sum reproduces conj(p) q of Gaussian data far inside
  the 1e-9 bound.
"""

import numpy as np

F16 = dict(bits=[8, 9, 9, 9], pairs_max=5, rows_per_flush=64)   # complex rows
I8 = dict(nsl=5, radix=128, pairs_max=6, rows_per_flush=32768)


def colscale_f16(col_max):
    e = np.frexp(col_max)[1]          # col_max < 2^e
    return np.ldexp(1.0, -e)


def slices_f16(x):
    """x in (-1, 1) -> integer slices s_1..s_4 with weights 2^-(8 + 9 (s-1))."""
    out, r = [], x.copy()
    for s, b in enumerate(F16["bits"]):
        t = r * 2.0 ** b
        sig = np.rint(t)
        out.append(sig)
        r = t - sig
    return out, r


def recon_f16(sl):
    w, acc = 2.0 ** -8, 0.0
    for s, sig in enumerate(sl):
        acc = acc + sig * w
        if s + 1 < len(sl):
            w = w * 2.0 ** -F16["bits"][s + 1]
    return acc


def colscale_i8(col_max):
    e = np.frexp(col_max * 128.0 / 127.0)[1]
    return np.ldexp(1.0, -e)


def slices_i8(x):
    out, r = [], x.copy()
    for _ in range(I8["nsl"]):
        t = r * 128.0
        sig = np.clip(np.rint(t), -127, 127)
        out.append(sig)
        r = t - sig
    return out, r


def test_f16_slices_exact_and_in_range():
    rng = np.random.default_rng(0)
    X = rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 8, 20000)
    X = np.concatenate([X, [np.max(np.abs(X))], [-np.max(np.abs(X))]])
    x = X * colscale_f16(np.max(np.abs(X)))
    assert np.all(np.abs(x) < 1)
    sl, r = slices_f16(x)
    assert np.all(np.abs(sl[0]) <= 256)
    for sig in sl[1:]:
        assert np.all(np.abs(sig) <= 256)
    for sig in sl:
        assert np.array_equal(sig.astype(np.float16).astype(np.float64), sig)
    # remainder below 2^-(8 + 27 + 1) of the column maximum
    assert np.max(np.abs(x - recon_f16(sl))) <= 2.0 ** -36 * (1 + 1e-12)


def test_i8_slices_exact_and_in_range():
    rng = np.random.default_rng(1)
    X = rng.standard_normal(20000)
    X[7] = 1.0                         # column max a power of two
    X[8] = -np.nextafter(1.0, 2.0)     # just above one
    m = np.max(np.abs(X))
    x = X * colscale_i8(m)
    assert np.all(np.abs(x) < 127 / 128)
    sl, r = slices_i8(x)
    assert np.all(np.abs(sl[0]) <= 127)
    for sig in sl[1:]:
        assert np.all(np.abs(sig) <= 64)
    for sig in sl:
        assert np.array_equal(sig.astype(np.int8).astype(np.float64), sig)
    rec = sum(sig * 128.0 ** -(s + 1) for s, sig in enumerate(sl))
    assert np.max(np.abs(x - rec)) <= 0.5 * 128.0 ** -5 * (1 + 1e-12)


def test_f16_leading_levels_exact_over_a_flush():
    # worst case: every interleaved real value at the top of its slice range
    n_real = 2 * F16["rows_per_flush"]
    lvl2 = n_real * 256 * 256                       # one pair (1, 1)
    lvl3 = n_real * 2 * 256 * 256                   # pairs (1, 2), (2, 1): |s_2| <= 2^8
    assert lvl2 <= 2 ** 24 and lvl3 <= 2 ** 24


def test_i8_levels_exact_over_a_flush():
    n_real = 2 * I8["rows_per_flush"]
    bound = {}
    for c in range(2, I8["pairs_max"] + 1):
        tot = 0
        for s in range(1, c):
            t = c - s
            if s > I8["nsl"] or t > I8["nsl"]:
                continue
            tot += (127 if s == 1 else 64) * (127 if t == 1 else 64)
        bound[c] = tot
    assert max(bound.values()) == 28544
    assert n_real * max(bound.values()) < 2 ** 31


def _split_dot(p, q, form):
    """Re/Im of sum_k conj(p_k) q_k from the truncated level sums."""
    if form == "f16":
        sp, sq = colscale_f16(np.max(np.abs(np.r_[p.real, p.imag]))), \
            colscale_f16(np.max(np.abs(np.r_[q.real, q.imag])))
        Pr, _ = slices_f16(p.real * sp)
        Pi, _ = slices_f16(p.imag * sp)
        Qr, _ = slices_f16(q.real * sq)
        Qi, _ = slices_f16(q.imag * sq)
        w = lambda s, t: 2.0 ** -(16 + 9 * (s + t))        # noqa: E731
        npair = 3                                           # s + t <= 3 (0-based) i.e. <= 5
    else:
        sp, sq = colscale_i8(np.max(np.abs(np.r_[p.real, p.imag]))), \
            colscale_i8(np.max(np.abs(np.r_[q.real, q.imag])))
        Pr, _ = slices_i8(p.real * sp)
        Pi, _ = slices_i8(p.imag * sp)
        Qr, _ = slices_i8(q.real * sq)
        Qi, _ = slices_i8(q.imag * sq)
        w = lambda s, t: 128.0 ** -(s + t + 2)             # noqa: E731
        npair = 4                                           # s + t <= 4 (0-based) i.e. <= 6
    re = im = 0.0
    for s in range(len(Pr)):
        for t in range(len(Qr)):
            if s + t > npair:
                continue
            re += w(s, t) * (np.dot(Pr[s], Qr[t]) + np.dot(Pi[s], Qi[t]))
            im += w(s, t) * (np.dot(Pr[s], Qi[t]) - np.dot(Pi[s], Qr[t]))
    return complex(re, im) / (sp * sq)


def test_truncated_products_within_bound():
    rng = np.random.default_rng(2)
    for form in ("f16", "i8"):
        errs = []
        for _ in range(20):
            p = rng.standard_normal(4000) + 1j * rng.standard_normal(4000)
            q = rng.standard_normal(4000) + 1j * rng.standard_normal(4000)
            exact = np.vdot(p, q)
            errs.append(abs(_split_dot(p, q, form) - exact) / abs(exact))
        # relative to |conj(p).q| ~ sqrt(n); the Frobenius bound the GPU
        # tests use is 1e-9
        assert np.median(errs) < 1e-9, (form, np.median(errs))
