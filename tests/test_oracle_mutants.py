"""Plausible mistakes planted in the CPU oracle (on the CPU only) must each
fail one of its pins: the pins are strong enough to catch them.

Each mutant replaces one oracle function (or a helper it calls) for the
duration of one test and runs the pin that is meant to catch it.
"""

import numpy as np
import pytest

import oracle
import oracle.ivfpq as ov
import test_oracle_pins as pins


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(ov, name, fn)
    monkeypatch.setattr(oracle, name, fn, raising=False)


def _adaptive(sel):
    """adaptive_params with one step replaced by `sel` (a mistake)."""
    def fn(scores, nprobe_max, metric, nprobe_init, nprobe_min, reorder_min, R, k, p0, p1):
        P = ov.select_probes(scores, nprobe_max)
        K = max(1, min(int(nprobe_init), int(nprobe_max)))
        row, K, rmin = sel(scores, P, K, int(nprobe_init), int(reorder_min), int(R), int(k))
        p = ov.hardness(row, K, metric)
        npb = ov.eq2(p, nprobe_min, nprobe_max, p0, p1)
        reo = ov.eq2(p, rmin, R, p0, p1)
        return npb, reo, p
    return fn


def _ok_rmin(reorder_min, R, k):
    return max(k, min(reorder_min, R))


ADAPTIVE_MUTANTS = {
    # the score row in list order instead of sorted by (score, list)
    "unsorted row": lambda s, P, K, ni, rm, R, k: (s, K, _ok_rmin(rm, R, k)),
    # nprobe_init not clamped to nprobe_max (over the whole sorted row)
    "K unclamped": lambda s, P, K, ni, rm, R, k: (s[ov.select_probes(s, len(s))], ni,
                                                 _ok_rmin(rm, R, k)),
    # the K-th nearest off by one either way
    "K - 1": lambda s, P, K, ni, rm, R, k: (s[P], max(1, K - 1), _ok_rmin(rm, R, k)),
    "K + 1": lambda s, P, K, ni, rm, R, k: (s[P], min(len(P), K + 1), _ok_rmin(rm, R, k)),
    # reorder_min not raised to k
    "rmin unclamped": lambda s, P, K, ni, rm, R, k: (s[P], K, min(rm, R)),
}


@pytest.mark.parametrize("name", sorted(ADAPTIVE_MUTANTS))
def test_adaptive_mutant_fails_its_pin(monkeypatch, name):
    _patch(monkeypatch, "adaptive_params", _adaptive(ADAPTIVE_MUTANTS[name]))
    with pytest.raises(AssertionError):
        pins.test_adaptive_params_hand_worked()


def test_adaptive_unmutated_passes():
    _adaptive(lambda s, P, K, ni, rm, R, k: (s[P], K, _ok_rmin(rm, R, k)))
    pins.test_adaptive_params_hand_worked()


@pytest.mark.parametrize("order", ["sequential", "reversed"])
def test_lo_sum_order_mutant_fails_its_pin(monkeypatch, order):
    def wrong(terms):
        t = np.asarray(terms, dtype=np.float32)
        return ov.seq_sum(t if order == "sequential" else t[..., ::-1])
    monkeypatch.setattr(ov, "tree_sum", wrong)
    with pytest.raises(AssertionError):
        pins.test_hand_worked_pairwise_lo_sum()


def _requantised(rounding):
    """quantize_lut with the entries rounded by `rounding` instead of rint."""
    real = ov.quantize_lut

    def fn(T, bias):
        q8, lo, delta, B = real(T, bias)
        D = np.asarray(T, dtype=np.float32) - lo[:, None]
        rng = D.max()
        if rng > 0:
            x = D * (np.float32(255) / rng)
            q8 = np.minimum(np.float32(255), rounding(x)).astype(np.uint8)
        return q8, lo, delta, B
    return fn


def test_half_up_rounding_fails_the_worked_example(monkeypatch):
    # Ties of i^2 / 2 go to the even neighbour; half-up moves them.
    _patch(monkeypatch, "quantize_lut", _requantised(lambda x: np.floor(x + np.float32(0.5))))
    with pytest.raises(AssertionError):
        pins.test_hand_worked_lut_example()


def test_floor_rounding_fails_the_error_bound(monkeypatch):
    # Truncation errs by up to delta per subspace, beyond m * delta / 2.
    _patch(monkeypatch, "quantize_lut", _requantised(np.floor))
    with pytest.raises(AssertionError):
        pins.test_quantisation_error_bound("c1")
