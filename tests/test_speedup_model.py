"""Host-side power-law speedup model (Section 5): the fit recovers a known law."""
import math

import numpy as np
import pytest

from paper_2303_16999_amd import speedup_model as SM


def test_fit_recovers_exact_power_law():
    law = {"a": 0.002, "alpha": 0.6, "beta": -0.5, "gamma": 0.45}
    pts = [(m, 1.0 / dd, b, SM.predict(m, 1.0 / dd, b, law))
           for m in (256, 1024, 4096, 8192) for dd in (4, 8, 16, 32) for b in (1, 4, 16)]
    f = SM.fit(pts)
    for key in ("alpha", "beta", "gamma"):
        assert abs(f[key] - law[key]) < 1e-9
    assert abs(f["a"] / law["a"] - 1.0) < 1e-9
    assert f["r2"] == pytest.approx(1.0)


def test_fit_with_noise_stays_close():
    rng = np.random.default_rng(0)
    law = {"a": 0.01, "alpha": 0.3, "beta": -0.8, "gamma": 0.2}
    pts = [(m, 1.0 / dd, b, SM.predict(m, 1.0 / dd, b, law) * math.exp(rng.normal(0, 0.05)))
           for m in (256, 512, 1024, 2048, 4096, 8192) for dd in (4, 8, 16, 32) for b in (1, 4, 8, 16)]
    f = SM.fit(pts)
    assert abs(f["alpha"] - 0.3) < 0.03 and abs(f["beta"] + 0.8) < 0.03 and abs(f["gamma"] - 0.2) < 0.03
    assert 0.04 < f["rms_log_error"] < 0.06


def test_paper_fit_values():
    # the paper's law at its base configuration m = 4096, d = 1/16, b = 16 (Section 5)
    assert SM.predict(4096, 1 / 16, 16) == pytest.approx(0.0013 * 4096 ** 0.59 * 16 ** 0.54 * 4.0)
    assert SM.predict(4096, 1 / 16, 16) > 1.0
    # unstructured, dense-ish and small: no speedup predicted
    assert SM.predict(256, 1 / 4, 1) < 1.0


def test_fit_rejects_too_few_points():
    with pytest.raises(ValueError):
        SM.fit([(256, 0.25, 1, 1.0)])


def test_library_model_matches_the_fit_constants():
    from paper_2303_16999_amd import spmm
    for m, d, b in ((256, 0.25, 1), (4096, 1 / 16, 16), (8192, 1 / 32, 8)):
        assert spmm.speedup_model(m, d, b) == pytest.approx(SM.predict(m, d, b, SM.MI355X_FIT), rel=1e-12)
    with pytest.raises(spmm.SpmmError):
        spmm.speedup_model(1024, 0.0, 16)
    with pytest.raises(spmm.SpmmError):
        spmm.speedup_model(0, 0.5, 16)
