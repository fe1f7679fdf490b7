"""The comparators the GPU parity tests use, checked on the CPU: they accept
every valid answer (any copy of a repeated key may be the one reported new
within its call) and reject plausible wrong ones."""
import numpy as np
import pytest

from oracle import first_occurrence_flags
from parity import check_flags_r2, check_flags_r2_calls


def _seq():
    rng = np.random.default_rng(0)
    return rng.integers(0, 50, size=400).astype(np.uint64)


BOUNDS = list(range(0, 400, 64)) + [400]


def _swap_winner(seq, ora, same_call):
    g = ora.copy()
    for k in np.unique(seq):
        idx = np.flatnonzero(seq == k)
        if len(idx) > 1 and ((idx[0] // 64 == idx[1] // 64) == same_call):
            j = idx[1] if same_call else idx[-1]
            g[idx[0]], g[j] = 0, 1
            return g
    raise AssertionError("no such key")


def test_calls_comparator_accepts_valid_answers():
    seq = _seq()
    ora = first_occurrence_flags(seq)
    check_flags_r2_calls(seq, ora, ora, BOUNDS)
    check_flags_r2_calls(seq, _swap_winner(seq, ora, True), ora, BOUNDS)   # another copy, same call
    check_flags_r2(seq, _swap_winner(seq, ora, True), ora)


@pytest.mark.parametrize("mistake", ["other_call", "extra_new", "missing_new", "flag_2", "twice"])
def test_calls_comparator_rejects_wrong_answers(mistake):
    seq = _seq()
    ora = first_occurrence_flags(seq)
    g = ora.copy()
    if mistake == "other_call":
        g = _swap_winner(seq, ora, False)
    elif mistake == "extra_new":
        g[np.flatnonzero(ora == 0)[0]] = 1
    elif mistake == "missing_new":
        g[np.flatnonzero(ora == 1)[3]] = 0
    elif mistake == "flag_2":
        g[np.flatnonzero(ora == 1)[3]] = 2
    else:                                       # two copies of one key reported new, one dropped elsewhere
        k = next(k for k in np.unique(seq) if (seq == k).sum() > 1)
        g[np.flatnonzero(seq == k)[1]] = 1
        g[np.flatnonzero((ora == 1) & (seq != k))[0]] = 0
    with pytest.raises(AssertionError):
        check_flags_r2_calls(seq, g, ora, BOUNDS)
