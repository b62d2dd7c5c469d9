"""The seeded input recipes (no cipher arithmetic)."""
import numpy as np

from paper_1909_04750_amd import synth


def test_splitmix64_published_values():
    # first outputs of splitmix64 for seeds 0 and 1234567 (reference sequence values)
    assert int(synth.draws(0, 0)) == 0xE220A8397B1DCDAF
    assert int(synth.draws(1234567, 0)) == 6457827717110365317


def test_draws_are_pure_functions_of_index():
    a = synth.draws(9, np.arange(100, dtype=np.uint64))
    b = np.array([int(synth.draws(9, j)) for j in range(100)], dtype=np.uint64)
    assert (a == b).all()


def test_keys_ivs_subset_equals_full():
    k, v = synth.keys_ivs(2, 1000)
    idx = np.array([0, 1, 17, 999])
    ks, vs = synth.keys_ivs(2, 1000, idx)
    assert (k[idx] == ks).all() and (v[idx] == vs).all()
    hi = int(synth.draws(2, 0))
    assert k[0, :8].tobytes() == hi.to_bytes(8, "big")
    assert k[0, 8:].tobytes() == int(synth.draws(2, 1)).to_bytes(8, "big")[:2]


def test_mixed_iv_lengths():
    L = synth.iv_lengths_mixed(3, 1 << 14)
    vals, counts = np.unique(L, return_counts=True)
    assert vals.tolist() == [0, 32, 64, 80]
    assert (abs(counts - (1 << 12)) < 400).all()


def test_batch_recipe_ranges():
    keys, ivs, ivb, nbits = synth.batch_requests(4, 10000)
    assert keys.shape == (10000, 10) and ivs.shape == (10000, 10)
    assert ivb.min() == 0 and ivb.max() == 80
    assert (nbits % 32 == 0).all()
    assert nbits.min() >= 256 and nbits.max() < (1 << 24)
    # log-uniform: about a quarter of the requests above 2^20 bits
    frac = (nbits >= (1 << 20)).mean()
    assert 0.2 < frac < 0.3
    k2, v2, b2, n2 = synth.batch_requests(4, 10000, max_log2=16.0)
    assert (k2 == keys).all() and (b2 == ivb).all() and n2.max() < (1 << 16)
