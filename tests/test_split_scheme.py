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


# ---------------------------------------------------------------------------
# Modular (CRT) INT8 form: each operand column is rounded to a signed b-bit
# integer at its column scale; the exact integer products are computed modulo
# eleven pairwise coprime moduli <= 255 on INT8 MFMA (symmetric residues, so
# every residue and its negation fit int8) and rebuilt by mixed-radix
# (Garner) reconstruction. Model written from the definitions (Chinese
# remainder theorem, Garner's algorithm), not shared with the HIP code.

CRT_MODULI = [255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217]
CRT_BMAX = 36


def crt_product():
    M = 1
    for m in CRT_MODULI:
        M *= m
    return M


def crt_bits(K):
    """Largest b (<= CRT_BMAX) with 2 K (2^(b-1))^2 <= (M - 1) / 2: every
    real or imaginary part of a K-row product of b-bit integers is then
    inside the symmetric residue range of M."""
    M = crt_product()
    b = CRT_BMAX
    while 2 * K * (1 << (2 * (b - 1))) > (M - 1) // 2:
        b -= 1
    return b


def sym_mod(x, m):
    r = x % m
    return np.where(r > m // 2, r - m, r) if isinstance(r, np.ndarray) else (r - m if r > m // 2 else r)


def crt_integers(X, b):
    """Column scale 2^-e (max < 2^e) and rint(x 2^(b-1)) of the scaled parts."""
    mx = np.max(np.maximum(np.abs(X.real), np.abs(X.imag)), axis=0)
    e = np.where(mx > 0, np.frexp(mx)[1], 0)
    sc = np.ldexp(1.0, b - 1 - e)
    return np.rint(X.real * sc).astype(np.int64), np.rint(X.imag * sc).astype(np.int64), e


def garner(res):
    """Symmetric residues r_i (lists per modulus) -> the integer in
    (-(M-1)/2, (M-1)/2) with those residues, by mixed radix digits."""
    v = []
    for i, m in enumerate(CRT_MODULI):
        t = int(res[i])
        for j in range(i):
            t = sym_mod((t - v[j]) * pow(CRT_MODULI[j], -1, m), m)
        v.append(sym_mod(t, m))
    x, w = 0, 1
    for i, m in enumerate(CRT_MODULI):
        x += v[i] * w
        w *= m
    return x, v


def test_crt_moduli_coprime_and_bit_budget():
    from math import gcd
    for i, a in enumerate(CRT_MODULI):
        assert a % 2 == 1 and a <= 255
        for c in CRT_MODULI[:i]:
            assert gcd(a, c) == 1
    M = crt_product()
    assert 86 < np.log2(float(M)) < 87
    assert crt_bits(8100) == 36 and crt_bits(25088) == 36
    assert crt_bits(1 << 17) == 34
    # symmetric residues of any modulus fit int8 with their negation
    assert max((m - 1) // 2 for m in CRT_MODULI) == 127
    # INT32 accumulation of residue products stays exact over the fold
    # interval of the kernel (65536 complex rows = 2^17 real products)
    assert (1 << 17) * 127 * 127 + 127 < 2 ** 31


def test_crt_reconstruction_exact():
    rng = np.random.default_rng(5)
    M = crt_product()
    half = (M - 1) // 2
    cases = [0, 1, -1, half, -half, half - 12345, -(half - 999)]
    cases += [int(x) for x in rng.integers(-2 ** 62, 2 ** 62, 50)]
    cases += [int(rng.integers(-2 ** 40, 2 ** 40)) * int(rng.integers(1, 2 ** 45)) for _ in range(50)]
    for x in cases:
        res = [sym_mod(x, m) for m in CRT_MODULI]
        assert all(abs(r) <= 127 for r in res)
        y, v = garner(res)
        assert y == x
        assert all(abs(d) <= (m - 1) // 2 for d, m in zip(v, CRT_MODULI))


def _garner_tables():
    """w[i][j] = W_j mod m_i, u[i] = W_i^-1 mod m_i, wu = w u mod m_i (symmetric)."""
    n = len(CRT_MODULI)
    w = [[0] * n for _ in range(n)]
    wu = [[0] * n for _ in range(n)]
    u = [0] * n
    for i, mi in enumerate(CRT_MODULI):
        wm = 1
        for j in range(i):
            w[i][j] = sym_mod(wm, mi)
            wm = wm * CRT_MODULI[j] % mi
        u[i] = sym_mod(pow(wm, -1, mi), mi)
        for j in range(i):
            wu[i][j] = sym_mod(w[i][j] * u[i], mi)
    return w, u, wu


def _garner_f32(rbytes):
    """The reconstruction's arithmetic as the kernel does it, in float32 (every
    product and sum is an integer below 2^24, so fused and unfused forms
    agree) and float64: digits, groups of three, Horner."""
    _, u, wu = _garner_tables()
    f = np.float32
    v = [f(rbytes[0]) - f(127)]
    for i in range(1, len(CRT_MODULI)):
        mi = f(CRT_MODULI[i])
        inv = f(1) / mi
        s = f(rbytes[i]) * f(u[i]) - f(127) * f(u[i])
        assert abs(float(s)) < 2 ** 24
        for j in range(i):
            s = s - f(wu[i][j]) * v[j]
            assert abs(float(s)) < 2 ** 24
        v.append(s - mi * np.rint(s * inv))
    m = [f(x) for x in CRT_MODULI]
    g = [float(v[i] + m[i] * (v[i + 1] + m[i + 1] * v[i + 2])) for i in (0, 3, 6)]
    g.append(float(v[9] + m[9] * v[10]))
    assert all(abs(x) < 2 ** 24 for x in g)
    P3 = float(CRT_MODULI[0] * CRT_MODULI[1] * CRT_MODULI[2])
    P6 = float(CRT_MODULI[3] * CRT_MODULI[4] * CRT_MODULI[5])
    P9 = float(CRT_MODULI[6] * CRT_MODULI[7] * CRT_MODULI[8])
    return ((g[3] * P9 + g[2]) * P6 + g[1]) * P3 + g[0], [int(x) for x in v]


def test_crt_garner_digits_in_float32():
    """The kernel's FP32 digits equal the exact mixed-radix digits, and its
    FP64 value is the integer up to the rounding of the last few steps."""
    rng = np.random.default_rng(9)
    M = crt_product()
    half = (M - 1) // 2
    cases = [0, 1, -1, half, -half, 127, -(half - 5)]
    cases += [int(x) for x in rng.integers(-2 ** 62, 2 ** 62, 200)]
    cases += [int(rng.integers(-2 ** 43, 2 ** 43)) * int(rng.integers(1, 2 ** 42)) for _ in range(200)]
    for x in cases:
        rbytes = [sym_mod(x, m) + 127 for m in CRT_MODULI]
        assert all(0 <= r <= 254 for r in rbytes)
        got, digits = _garner_f32(rbytes)
        _, exact_digits = garner([r - 127 for r in rbytes])
        assert digits == exact_digits
        assert abs(got - x) <= 2.0 ** -50 * max(abs(x), 1)


def _crt_dot_columns(P, Q, b):
    """conj(P)^T Q through the modular form, exactly as the kernels define it."""
    Pr, Pi, eP = crt_integers(P, b)
    Qr, Qi, eQ = crt_integers(Q, b)
    n, k = P.shape[1], Q.shape[1]
    out = np.zeros((n, k), complex)
    for g in range(n):
        for h in range(k):
            re_res, im_res = [], []
            for m in CRT_MODULI:
                pr, pi = sym_mod(Pr[:, g], m), sym_mod(Pi[:, g], m)
                qr, qi = sym_mod(Qr[:, h], m), sym_mod(Qi[:, h], m)
                # INT32 sums of residue products, then reduced
                re_res.append(sym_mod(int(np.dot(pr, qr) + np.dot(pi, qi)), m))
                im_res.append(sym_mod(int(np.dot(pr, qi) - np.dot(pi, qr)), m))
            xr, _ = garner(re_res)
            xi, _ = garner(im_res)
            # exact integer products (Python integers: they exceed int64)
            pr_, pi_ = Pr[:, g].astype(object), Pi[:, g].astype(object)
            qr_, qi_ = Qr[:, h].astype(object), Qi[:, h].astype(object)
            exact_r = int(np.dot(pr_, qr_) + np.dot(pi_, qi_))
            exact_i = int(np.dot(pr_, qi_) - np.dot(pi_, qr_))
            assert (xr, xi) == (exact_r, exact_i)
            w = np.ldexp(1.0, int(eP[g] + eQ[h]) - 2 * (b - 1))
            out[g, h] = complex(float(xr) * w, float(xi) * w)
    return out


def test_crt_products_exact_and_within_bound():
    rng = np.random.default_rng(6)
    K = 3000
    b = crt_bits(K)
    P = (rng.standard_normal((K, 3)) + 1j * rng.standard_normal((K, 3))) * np.array([1.0, 1e-3, 1e5])
    Q = (rng.standard_normal((K, 2)) + 1j * rng.standard_normal((K, 2))) * np.array([3.0, 1e-7])
    P[5, 0] = 2.0 ** 3          # a column maximum that is a power of two
    got = _crt_dot_columns(P, Q, b)
    ref = P.conj().T @ Q
    err = np.abs(got - ref) / (np.linalg.norm(P, axis=0)[:, None] * np.linalg.norm(Q, axis=0)[None, :])
    # rounding both operands to b bits of their column maxima: far inside
    # the 1e-9 bound of the split forms
    assert np.max(err) < 2.0 ** -(b - 4)
