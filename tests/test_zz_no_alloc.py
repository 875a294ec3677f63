"""The allocation-free entry point pic_fields_noalloc against pic_fields
(the same deposit, Poisson and cell kernels; scratch in a file-scope device
array instead of a workspace): two calls in a row, the second smaller, each
compared with pic_fields on the same input (cells bit for bit, the charge at
1e-12 and the potential and field at 1e-10 relative: the LDS double atomics
of the deposit make the charge reproducible to rounding only)."""
import numpy as np
import pytest

from workloads import make_ensemble, workload

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_noalloc_matches_pic_fields_on_two_calls():
    import torch
    from paper_2201_05555_amd import binding
    assert torch.cuda.is_available()
    for kw in (dict(N=30001, p=24, Nx=128), dict(N=777, p=5, Nx=48)):
        print("[case] pic_fields_noalloc", kw, flush=True)
        w = workload("twostream_deim", **kw)
        e = make_ensemble(w)
        X = e["X0"] + np.outer(np.linspace(-2, 2, e["X0"].shape[0]), e["L"])
        c0, r0, P0, e0 = binding.pic_fields(X, e["L"], w["Nx"])
        c1, r1, P1, e1 = binding.pic_fields_noalloc(X, e["L"], w["Nx"])
        torch.cuda.synchronize()
        assert torch.equal(c0, c1)
        assert _rel(r1.cpu().numpy(), r0.cpu().numpy()) < 1e-12
        assert _rel(P1.cpu().numpy(), P0.cpu().numpy()) < 1e-10
        assert _rel(e1.cpu().numpy(), e0.cpu().numpy()) < 1e-10


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    from paper_2201_05555_amd import binding
    assert torch.cuda.is_available()
    p, Nx, N = 1000, 1000, 1000
    X = torch.zeros((p, N), dtype=torch.float64, device="cuda")
    with pytest.raises(binding.SymromError) as ei:
        binding.pic_fields_noalloc(X, np.full(p, 2 * np.pi), Nx)
    assert ei.value.status == binding.EINVAL
