"""Pins of the oracle's feature switches (the ablation of Sec. VI-B, Table IV).

The base configuration is the cuSZp-equivalent compressor: first-order
Lorenzo on independent 32-element blocks, no centering.  +Cross adds the
cross-block prediction state, +Cent adaptive centering, +LZ2 the second
order (= the full method).  Checked against facts outside the oracle:
the independent-block rates of Fig. 2 (tests/golden), a brute-force Python
evaluation of every variant under every switch setting, an independent
Python encoder, the variant-set inclusions (a minimum over a superset of
variants can only be smaller), and the reconstruction, which depends on the
quantized values alone and so must be bit-identical under every setting.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import workloads
from tests import fsz_format as fmt
from tests.test_oracle import _fields, _tiny_tiles, golden, unit_grid

FEATURES = list(range(8))
BASE, CROSS, CROSS_CENT, FULL = 0, 1, 3, 7


def test_fig2_independent_block_rates():
    """Fig. 2: with independent blocks the raw boundary values 1000, 1008,
    1024 are the first residuals and the blocks need rate 10-11; the
    cross-block state brings them to 1."""
    g = golden("fig2_cross_block.json")
    q = np.concatenate([g["start"][b] + np.arange(32) // g["step"][b] for b in range(8)])
    x, _, _, inv = unit_grid(q)
    _, _, _, r_base, _ = oracle.tile_eval_features(x, inv, BASE)
    _, _, _, r_cross, _ = oracle.tile_eval_features(x, inv, CROSS)
    for k, b in enumerate(g["blocks_checked"]):
        assert r_base[0][b] == g["independent_rates"][k]
        assert r_cross[0][b] == g["cross_block_rate"]


@pytest.mark.parametrize("features", FEATURES)
def test_features_bruteforce_tiles(features):
    rng = np.random.default_rng(31 + features)
    for q in _tiny_tiles(rng):
        x, eb, E, inv = unit_grid(q)
        mu_bf, ok_bf, cost_bf, rates_bf, best_bf = fmt.brute_force_tile(x, inv, features)
        mu, ok, cost, rates, best = oracle.tile_eval_features(x, inv, features)
        assert (mu, ok) == (mu_bf, ok_bf)
        assert list(cost) == cost_bf
        assert rates.tolist() == rates_bf
        assert best == best_bf


@pytest.mark.parametrize("features", FEATURES)
def test_features_stream_matches_python_encoder(features):
    rng = np.random.default_rng(40 + features)
    for n in (1, 33, 256, 300, 513, 2048 + 77):
        q = np.cumsum(rng.integers(-4, 5, n)) + rng.integers(-300, 300)
        x, eb, E, inv = unit_grid(q)
        choices = []
        for t in range(fmt.ceil_div(n, 256)):
            mu, _, _, _, best = fmt.brute_force_tile(x[t * 256:(t + 1) * 256], inv, features)
            choices.append((best & 1, best >> 1, mu))
        flags = 0 if features & fmt.CROSS_BLOCK else 2
        ref = fmt.encode_stream(x, E, inv, oracle.ABS, eb, flags, choices)
        s = oracle.compress(x, oracle.ABS, eb, features=features)
        assert s == ref
        assert np.array_equal(oracle.decompress(s, n).view(np.uint32),
                              fmt.closed_form(x, E, inv).view(np.uint32))


@pytest.mark.parametrize("name,x", list(_fields()))
def test_feature_inclusions_and_identical_reconstruction(name, x):
    for rel in (1e-2, 1e-3, 1e-4):
        if oracle.compress_status(x, oracle.REL, rel)[0] == oracle.ERR_EB_TOO_SMALL:
            continue  # no binary32 grid honours this bound (rejected in every setting)
        size = {}
        recon = None
        for f in FEATURES:
            s = oracle.compress(x, oracle.REL, rel, features=f)
            size[f] = len(s)
            y = oracle.decompress(s, x.size)
            if recon is None:
                recon = y
            assert np.array_equal(y.view(np.uint32), recon.view(np.uint32)), (name, rel, f)
            hdr = fmt.parse_header(s)
            assert (hdr["flags"] >> 1) & 1 == (0 if f & fmt.CROSS_BLOCK else 1)
        # per tile the selection is a minimum over the allowed variants, so a
        # setting whose allowed set contains another's (same block structure)
        # can only be smaller
        for cross in (0, fmt.CROSS_BLOCK):
            for a, b in itertools.product(range(4), repeat=2):
                fa, fb = cross | (a << 1), cross | (b << 1)
                if (a & b) == b:  # fa allows everything fb allows
                    assert size[fa] <= size[fb], (name, rel, fa, fb)
        # the full method is the ablation's last column
        assert size[FULL] == len(oracle.compress(x, oracle.REL, rel))


def test_base_sizes_closed_form():
    """Base (LZ1, independent blocks): block rate = bit length of the largest
    of |q0| and the in-block first differences, from numpy alone."""
    for n, seed in ((1000, 3), (4096 + 19, 5), (300, 7)):
        x = workloads.sinusoid_field(n, seed)
        st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
        q = fmt.quantize(x, inv)
        total = fmt.data_start(n)
        for b in range(0, n, 32):
            blk = q[b:b + 32]
            a = max(abs(int(blk[0])), int(np.abs(np.diff(blk)).max()) if blk.size > 1 else 0)
            total += fmt.block_cost(fmt.bitlen(a))
        assert len(oracle.compress(x, oracle.REL, 1e-3, features=BASE)) == total


def test_independent_ragged_round_trips():
    for n in (1, 2, 31, 32, 33, 255, 257, 1000):
        x = workloads.sinusoid_field(n, n)
        for f in (BASE, fmt.CENTERING | fmt.LZ2):
            s = oracle.compress(x, oracle.REL, 1e-3, features=f)
            st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
            y = oracle.decompress(s, n)
            assert np.array_equal(y.view(np.uint32), fmt.closed_form(x, E, inv).view(np.uint32))


def test_invalid_feature_bits():
    x = workloads.sinusoid_field(100, 1)
    assert oracle.compress_status(x, oracle.REL, 1e-3, features=8)[0] == oracle.ERR_INVALID_ARG
