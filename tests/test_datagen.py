"""Host checks of datagen's exactly reproducible fields: the signal does not depend on
the summation order (so a GPU loop and a host BLAS product agree bit for bit), the
counter-based noise follows its definition and statistics, and terms switch on as
specified."""

import numpy as np

import datagen


def small_spec(**kw):
    args = dict(grid=(7, 6, 5), channels=3, terms=6, N=3, n_batches=4, drift=1e-3, seed=11, batch_seed0=110,
                nu=1e-6)
    args.update(kw)
    return datagen.FieldSpec(**args)


def test_signal_is_exact_in_any_order():
    ff = datagen.exact_field_factors(small_spec(), 2)
    T, N, P1 = ff.A.shape
    for s in range(N):
        blas = ff.A[:, s, :].T @ ff.B
        fwd = np.zeros_like(blas)
        for t in range(T):
            fwd = fwd + ff.A[t, s, :, None] * ff.B[t, None, :]
        rev = np.zeros_like(blas)
        for t in reversed(range(T)):
            rev = rev + ff.A[t, s, :, None] * ff.B[t, None, :]
        assert np.array_equal(blas, fwd) and np.array_equal(fwd, rev)


def test_factors_are_24_bit_fixed_point():
    ff = datagen.exact_field_factors(small_spec(), 1)
    for X in (ff.A, ff.B):
        mx = np.max(np.abs(X))
        q = 2.0 ** (np.frexp(mx)[1] - datagen.FIXED_BITS)
        assert np.array_equal(np.round(X / q) * q, X)
        assert np.max(np.abs(X / q)) <= 2 ** datagen.FIXED_BITS


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    out = datagen.splitmix64(np.arange(3, dtype=np.uint64))
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_noise_statistics_and_exactness():
    g = datagen.noise_unit(123, 0, 1 << 20)
    assert abs(g.mean()) < 3e-3
    assert abs(g.var() - 1.0 / 3.0) < 3e-3
    # multiples of 2^-16 within the Irwin-Hall support
    assert np.array_equal(np.round(g * 65536.0), g * 65536.0)
    assert g.min() >= -2.0 and g.max() <= 2.0
    # counters are per element: a slice equals the same range of the whole
    np.testing.assert_array_equal(datagen.noise_unit(123, 1000, 50), g[1000:1050])


def test_terms_switch_on():
    spec = small_spec(active0=2, onset_every=3)
    assert list(datagen.term_mask(spec, 0)) == [1, 1, 0, 0, 0, 0]
    assert list(datagen.term_mask(spec, 3)) == [1, 1, 1, 0, 0, 0]
    assert list(datagen.term_mask(spec, 12)) == [1] * 6
    ff = datagen.exact_field_factors(spec, 0)
    assert np.all(ff.A[2:] == 0)


def test_host_batch_is_the_rounded_signal_plus_noise():
    spec = small_spec()
    ff = datagen.exact_field_factors(spec, 3)
    y = datagen.exact_field_batch(spec, 3).reshape(-1)
    sig = np.concatenate([(ff.A[:, s, :].T @ ff.B).reshape(-1) for s in range(spec.N)])
    g = datagen.noise_unit(ff.key, 0, sig.size)
    np.testing.assert_array_equal(y, (sig + ff.scale * g).astype(np.float32))
