"""The skewed and concentrated pattern generators (host only)."""
import numpy as np
import pytest

from paper_2303_16999_amd import synth


@pytest.mark.parametrize("mb,kb,d,alpha", [(512, 512, 1 / 16, 1.0), (64, 20, 0.5, 2.0), (100, 300, 0.01, 0.5),
                                           (33, 7, 1.0, 1.5)])
def test_skewed_mask_exact_count_and_power_law(mb, kb, d, alpha):
    M = synth.skewed_mask(mb, kb, d, alpha, seed=4)
    assert M.shape == (mb, kb) and M.dtype == np.uint8
    assert int(M.sum()) == synth.nnzb_for_density(mb, kb, d)
    counts = np.sort(M.sum(1))[::-1]
    assert counts.max() <= kb
    if d < 0.5 and mb >= 64:
        assert counts[0] >= 4 * max(1, counts[len(counts) // 2])  # a heavy head
    assert np.array_equal(M, synth.skewed_mask(mb, kb, d, alpha, seed=4))


@pytest.mark.parametrize("mb,kb,d", [(512, 512, 1 / 16), (10, 7, 0.35), (8, 8, 1.0)])
def test_concentrated_mask_fills_few_rows(mb, kb, d):
    M = synth.concentrated_mask(mb, kb, d, seed=2)
    nnzb = synth.nnzb_for_density(mb, kb, d)
    assert int(M.sum()) == nnzb
    assert int((M.sum(1) > 0).sum()) == -(-nnzb // kb)
    assert int((M.sum(1) == kb).sum()) == nnzb // kb
