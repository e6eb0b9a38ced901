"""Pins of the closure oracle (oracle.cnn): brute-force convolution, adjoint identities,
finite-difference gradients, the first Adam step and bfloat16 rounding."""
import numpy as np

from oracle import cnn

R = np.random.default_rng(7)


def test_bf16_rounding_known_values():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -7, 3.1415927, 0.0])
    r = cnn.bf16_round(v)
    # 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1.0);
    # 1 + 3 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert list(r[:5]) == [1.0, 1.0, 1.0 + 2 ** -6, -2.5, 1.0 + 2 ** -7]
    assert r[5] == 3.140625 and r[6] == 0.0


def test_conv_matches_explicit_loops():
    n, ci, co = 4, 2, 3
    x = R.standard_normal((ci, n, n, n))
    w = R.standard_normal((co, ci, 27))
    b = R.standard_normal(co)
    y = cnn.conv(x, w, b)
    ref = np.zeros_like(y)
    for o in range(co):
        for z in range(n):
            for yy in range(n):
                for xx in range(n):
                    s = b[o]
                    for c in range(ci):
                        for t, (dz, dy, dx) in enumerate(cnn.TAPS):
                            s += w[o, c, t] * x[c, (z + dz) % n, (yy + dy) % n, (xx + dx) % n]
                    ref[o, z, yy, xx] = s
    assert np.max(np.abs(y - ref)) < 1e-12


def test_adjoint_identities():
    n = 6
    x = R.standard_normal((4, n, n, n))
    w = R.standard_normal((5, 4, 27))
    dy = R.standard_normal((5, n, n, n))
    lhs = np.sum(dy * cnn.conv(x, w, None))
    assert abs(lhs - np.sum(cnn.conv_transpose(dy, w) * x)) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(cnn.conv_weight_grad(x, dy) * w)) < 1e-10 * abs(lhs)
    pos = R.random((300, 3))
    f = R.standard_normal((3, n, n, n))
    vals = R.standard_normal((300, 3))
    a = np.sum(vals * cnn.gather(f, pos))
    assert abs(a - np.sum(cnn.gather_adjoint(vals, pos, n) * f)) < 1e-10 * abs(a)


def test_gradients_against_finite_differences():
    n = 4
    x = R.standard_normal((4, n, n, n))
    p = 0.3 * R.standard_normal(cnn.N_PARAMS)
    p[cnn.N_PARAMS - 3:] = 0.0
    dy = R.standard_normal((3, n, n, n))

    def loss(q):
        return np.sum(dy * cnn.forward(q, x, emulate_bf16=False)[0])

    _, acts = cnn.forward(p, x, emulate_bf16=False)
    g = cnn.backward(p, acts, dy, emulate_bf16=False)
    for i in R.choice(cnn.N_PARAMS, 40, replace=False):
        h = 1e-6
        e = np.zeros_like(p)
        e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_first_adam_step_moves_by_lr_times_sign():
    r = np.random.default_rng(73)
    p = r.standard_normal(50)
    g = r.standard_normal(50)
    q, m, v = cnn.adam(p, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    # bias-corrected first step: lr g / (|g| + eps), i.e. lr sign(g) up to eps / |g|
    assert np.allclose(q - p, -1e-3 * np.sign(g), rtol=1e-8 / np.min(np.abs(g)) + 1e-12, atol=0)
    # the moments are the bias-uncorrected running averages
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_the_library_conversion():
    """Against an independent implementation: torch's float32 -> bfloat16 conversion (round to
    nearest, ties to even) on random values, exact ties, subnormals, infinities and signed zeros."""
    import torch
    r = np.random.default_rng(11)
    v = np.concatenate([
        r.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** r.integers(-30, 30, 20000).astype(np.float32),
        # exact ties: low 16 bits 0x8000 with both parities of the kept bit
        (r.integers(0, 2 ** 31, 4000, dtype=np.uint64).astype(np.uint32) & np.uint32(0xFFFF0000)
         | np.uint32(0x8000)).view(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 1e-40, -3e-39, 3.4e38], dtype=np.float32),
    ])
    v = v[np.isfinite(v) | np.isinf(v)]
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    got = cnn.bf16_round(v)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all(), v[~same][:5]
    assert np.array_equal(np.signbit(got), np.signbit(want))
