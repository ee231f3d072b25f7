"""MPSNR / MSSIM on the GPU (ifctn_image_metrics) against the oracle's plain
definitions.  Both sum in float64 from the same input values, so only the
summation order differs: relative agreement 1e-12."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2511_16358_amd import ifctn
    ifctn.lib()
    return ifctn


@pytest.mark.parametrize("shape,dtype", [((23, 19, 4), np.float64), ((23, 19, 4), np.float32),
                                         ((11, 11, 1), np.float64), ((40, 31, 7), np.float32)])
def test_metrics_match_oracle(shape, dtype):
    from paper_2511_16358_amd import ifctn
    rng = np.random.default_rng(sum(shape))
    ref = rng.uniform(0, 1, size=shape).astype(dtype)
    X = np.clip(ref + rng.normal(0, 0.08, size=shape), 0, 1).astype(dtype)
    mp, ms, ps, ss = ifctn.image_metrics(X, ref)
    X64, R64 = X.astype(np.float64), ref.astype(np.float64)
    ps_o = oracle.psnr_bands(X64, R64)
    ss_o = np.array([oracle.ssim_band(X64[:, :, b], R64[:, :, b]) for b in range(shape[2])])
    assert np.allclose(ps, ps_o, rtol=1e-12, atol=0)
    assert np.allclose(ss, ss_o, rtol=1e-12, atol=1e-14)
    assert abs(mp - oracle.mpsnr(X64, R64)) <= 1e-12 * abs(mp)
    assert abs(ms - oracle.mssim(X64, R64)) <= 1e-12 * abs(ms) + 1e-14


def test_identical_and_invalid():
    from paper_2511_16358_amd import ifctn
    ref = np.random.default_rng(0).uniform(0, 1, size=(12, 14, 2))
    mp, ms, ps, ss = ifctn.image_metrics(ref, ref)
    assert np.all(np.isinf(ps)) and np.allclose(ss, 1.0, atol=1e-14)
    with pytest.raises(ifctn.IfctnError) as e:
        ifctn.image_metrics(ref[:10], ref[:10])
    assert e.value.status == ifctn.IFCTN_E_INVAL


def test_msi256_sized_metrics_sampled_bands():
    """Full 256 x 256 x 31 size: every band's PSNR, and the SSIM of three
    sampled bands, against the oracle."""
    from paper_2511_16358_amd import ifctn
    rng = np.random.default_rng(7)
    ref = rng.uniform(0, 1, size=(256, 256, 31)).astype(np.float32)
    X = np.clip(ref + rng.normal(0, 0.05, size=ref.shape), 0, 1).astype(np.float32)
    mp, ms, ps, ss = ifctn.image_metrics(X, ref)
    X64, R64 = X.astype(np.float64), ref.astype(np.float64)
    assert np.allclose(ps, oracle.psnr_bands(X64, R64), rtol=1e-12, atol=0)
    for b in (0, 15, 30):
        assert abs(ss[b] - oracle.ssim_band(X64[:, :, b], R64[:, :, b])) <= 1e-12 * abs(ss[b])
    assert abs(ms - ss.mean()) < 1e-15 and abs(mp - ps.mean()) < 1e-12
