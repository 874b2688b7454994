"""The library's FIR design on the host (qtb_filter_taps, no device call)
against the oracle's independent design: theta of eq. (1) and kappa_P of
eq. (10-11) sampled on the FIR grid, taps by the inverse DFT of the square
root (two FP64 codes with different quadratures for kappa_P: 1e-12)."""
import numpy as np
import pytest

from paper_1905_02521_amd import qtb, workloads as W

U = W.METAL_UNITS


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(os.environ.get("QTB_LIB", qtb.LIB_PATH)):
        pytest.skip("libqtb.so not built")
    return qtb.lib()


@pytest.mark.parametrize("kind,P,T,two_nf", [(0, 1, 300.0, 2), (1, 1, 50.0, 512), (1, 1, 20.0, 2048),
                                             (2, 2, 100.0, 256), (2, 8, 50.0, 512),
                                             (2, 32, 50.0, 1024)])
def test_host_taps_match_oracle(lib, orc, kind, P, T, two_nf):
    h = qtb.qtb_filter_taps(kind, T, P, 1.0, two_nf, U["hbar"], U["kB"])
    o = orc.taps(kind, T, P, 1.0, two_nf, orc.make_units(**U))
    assert np.max(np.abs(h - o)) <= 1e-12 * np.max(np.abs(o))
    if kind == 0:  # white noise: sqrt(k_B T) at k = 0 only
        assert h[two_nf // 2] == pytest.approx(np.sqrt(U["kB"] * T), rel=1e-15)


@pytest.mark.parametrize("args", [
    (3, 50.0, 1, 1.0, 512), (1, 0.0, 1, 1.0, 512), (1, 50.0, 1, -1.0, 512), (2, 50.0, 0, 1.0, 512),
    (2, 50.0, 65, 1.0, 512), (1, 50.0, 1, 1.0, 500), (1, 50.0, 1, 1.0, 16384), (1, 50.0, 1, 1.0, 1)])
def test_host_taps_reject_bad_arguments(lib, args):
    with pytest.raises(qtb.QtbError) as e:
        qtb.qtb_filter_taps(*args, U["hbar"], U["kB"])
    assert e.value.status == qtb.QTB_E_INVALID
