"""The allocation-free spectrum entry point (qtb_vdos_spectrum_noalloc)
against the one that takes a workspace (qtb_vdos_spectrum): the same kernels
on the same series, so the spectra agree bit for bit, on two calls in a row
(the second with a smaller input, which reuses the static scratch that the
first left behind), and sizes beyond the static scratch are refused."""
import ctypes

import numpy as np
import pytest

from paper_1905_02521_amd import qtb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    qtb.lib()
    return t


def _series(torch, n_samples, n_dof, seed):
    g = torch.Generator().manual_seed(seed)
    v = torch.randn(n_samples, n_dof, dtype=torch.float64, generator=g).cuda()
    w = (0.5 + torch.rand(n_dof, dtype=torch.float64, generator=g)).cuda()
    return v, w


def test_noalloc_spectrum_equals_workspace_spectrum(torch):
    # first call: 6 segments of 512 samples, 3000 dofs (several FFT groups,
    # a ragged last group); second: fewer samples and dofs, a shorter segment
    for n_samples, n_dof, seg, seed in ((3072, 3000, 512, 1), (640, 77, 128, 2)):
        v, w = _series(torch, n_samples, n_dof, seed)
        ref = qtb.vdos_spectrum(v, w, seg)
        got = qtb.vdos_spectrum_noalloc(v, w, seg)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert a.shape == (seg // 2 + 1,)
        assert np.all(np.isfinite(b)) and np.any(b != 0.0)
        assert np.array_equal(a, b), np.max(np.abs(a - b))
    # dof-major series (the other stride order), into a caller's output
    v, w = _series(torch, 1024, 500, 3)
    vt = v.t().contiguous()
    out = torch.empty(129, dtype=torch.float64, device="cuda")
    qtb.vdos_spectrum_noalloc(vt, w, 256, dof_major=True, out=out)
    ref = qtb.vdos_spectrum(vt, w, 256, dof_major=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_spectrum_refuses_sizes_beyond_its_scratch(torch):
    L = qtb.lib()
    n_dof, seg = 4_000_000, 4096
    assert L.qtb_vdos_workspace_bytes(n_dof, seg, 0) > 16 << 20
    v = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = L.qtb_vdos_spectrum_noalloc(ctypes.c_void_p(v.data_ptr()), seg, n_dof, n_dof, 1,
                                     ctypes.c_void_p(v.data_ptr()), seg,
                                     ctypes.c_void_p(v.data_ptr()), None)
    assert st == qtb.QTB_E_INVALID
    assert b"static" in L.qtb_last_error(None)
