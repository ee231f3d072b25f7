"""ifctn_assemble_noalloc, the allocation-free assemble: through the C ABI it
must give exactly what ifctn_assemble gives (same kernels, same order, only
the staging memory differs) and the oracle's iFCTN(G) within the tolerances
of the assemble parity test, on two calls in a row, the second smaller, so
that nothing the first call left in the shared array leaks into the second."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2511_16358_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def _factors(dims, R, seed):
    ranks = W.uniform_ranks(len(dims), R)
    rng = np.random.default_rng(seed)
    G = {k: rng.standard_normal(s) for k, s in W.factor_shapes(dims, ranks)}
    return ranks, G


@pytest.mark.parametrize("precision,tol", [(2, 1e-12), (0, 1e-6)])
def test_noalloc_assemble_matches_assemble_twice(precision, tol):
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2511_16358_amd import ifctn
    ifctn.lib()
    # the first call is the larger: order 4 with ragged sizes, then order 3
    for call, (dims, R, seed) in enumerate([((37, 29, 11, 6), 4, 11), ((9, 13, 7), 3, 12)]):
        print(f"[case] noalloc call={call} dims={dims} R={R} precision={precision}", flush=True)
        ranks, G = _factors(dims, R, seed)
        want = ifctn.assemble(dims, ranks, G, precision=precision)
        out = torch.full(dims, float("nan"), dtype=want.dtype, device="cuda")
        got = ifctn.assemble(dims, ranks, G, precision=precision, out=out, noalloc=True)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, want), (call, float((got.double() - want.double()).abs().max()))
        assert relerr(got.cpu().numpy(), oracle.reconstruct(G, dims)) < tol


def test_noalloc_assemble_rejects_oversize():
    """A problem whose edge matrices exceed the fixed array is refused with
    IFCTN_E_UNSUPPORTED before any device work; the output is untouched."""
    from paper_2511_16358_amd import ifctn
    dims = (1200, 1200, 4)                  # W_01 alone: 1200^2 (8 + 4) bytes > 16 MiB
    ranks, G = _factors(dims, 2, 13)
    out = torch.zeros(dims, dtype=torch.float32, device="cuda")
    params = ifctn.make_params(dims, ranks, precision=ifctn.IFCTN_FP32)
    g = np.ascontiguousarray(W.pack(G, dims, ranks), dtype=np.float64)
    st = ifctn.lib().ifctn_assemble_noalloc(ctypes.byref(params),
                                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            ctypes.c_void_p(out.data_ptr()), None)
    assert st == ifctn.IFCTN_E_UNSUPPORTED
    assert "allocation-free" in ifctn.lib().ifctn_last_error().decode()
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out)) == 0
