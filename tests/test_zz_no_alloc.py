"""The allocation-free D apply (grg_dirac_apply_noalloc) against the
allocating one (grg_dirac_apply) through the C-ABI: same kernels and launch,
so the outputs must be identical bit for bit, over two and more calls in a
row on one GPU (each later call on a smaller input, so stale scratch contents
from the bigger call sit where the smaller one's padding is), in every
precision, with the oracle as the reference for the FP64 values; device
memory does not shrink across calls after the first; requests beyond the
scratch are refused with GRG_ETOO_LARGE."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import matfree

from gpu_support import Lattice, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-14, "fp32": 2e-6, "bf16": 1.5e-2}


def _both(lat, m0, prec, x, nrhs):
    import torch

    xd = to_dev(x)
    y_ref = torch.empty_like(xd)
    y_new = torch.full_like(xd, float("nan"))
    lat.grg.grg_dirac_apply(lat.h, m0, prec, xd, y_ref, nrhs)
    lat.grg.grg_dirac_apply_noalloc(lat.h, m0, prec, xd, y_new, nrhs)
    return to_host(y_ref), to_host(y_new)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_noalloc_matches_allocating_apply(prec):
    m0 = -0.2
    big = Lattice((8, 8, 8, 8), 0.5, 71)
    small = Lattice((6, 4, 4, 6), 0.5, 72)  # 576 sites: a ragged last tile
    calls = [(big, 4), (big, 1), (small, 3), (small, 1)]
    for i, (lat, nrhs) in enumerate(calls):
        print(f"noalloc call {i}: {lat.dims} nrhs {nrhs} {prec}", flush=True)
        x = gaussian_vectors(12 * lat.V, nrhs, 73 + i)
        ref, new = _both(lat, m0, prec, x, nrhs)
        assert np.array_equal(new, ref), (i, lat.dims, nrhs)
        want = matfree.dirac_apply(lat.links, lat.dims, m0, x)
        assert rel_err(new, want) < TOL[prec]
    big.close()
    small.close()


def test_noalloc_allocates_nothing():
    import torch

    m0 = 0.1
    lat = Lattice((8, 8, 8, 8), 0.5, 74)
    x = gaussian_vectors(12 * lat.V, 2, 74)
    xd = to_dev(x)
    y = torch.empty_like(xd)
    # the first call on the device looks up the scratch address
    lat.grg.grg_dirac_apply_noalloc(lat.h, m0, "fp64", xd, y, 2)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for prec in ("fp64", "bf16", "fp32", "fp64"):
        lat.grg.grg_dirac_apply_noalloc(lat.h, m0, prec, xd, y, 2)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0, (free0, free1)
    assert rel_err(to_host(y), matfree.dirac_apply(lat.links, lat.dims, m0, x)) < 1e-14
    lat.close()


def test_noalloc_too_large_is_refused():
    import torch

    grg = None
    lat = Lattice((16, 16, 16, 16), 0.5, 75)
    grg = lat.grg
    # 16^4 in FP64: 2 fields of 12.6 MB fit for one RHS, not for two
    x = to_dev(gaussian_vectors(12 * lat.V, 2, 75))
    y = torch.zeros_like(x)
    with pytest.raises(grg.GrgError) as ei:
        grg.grg_dirac_apply_noalloc(lat.h, -0.1, "fp64", x, y, 2)
    assert ei.value.status == grg.GRG_ETOO_LARGE
    assert not torch.any(y)  # nothing was enqueued
    # one RHS fits, and BF16 fits for more
    grg.grg_dirac_apply_noalloc(lat.h, -0.1, "fp64", x[:1], y[:1], 1)
    grg.grg_dirac_apply_noalloc(lat.h, -0.1, "bf16", x, y, 2)
    ref = torch.empty_like(x)
    grg.grg_dirac_apply(lat.h, -0.1, "bf16", x, ref, 2)
    assert torch.equal(y, ref)
    lat.close()
