"""Every stencil launch shape (site-parallel and t-marching, the shapes the
autotuner chooses between) against the oracle's sub-block applies
D_rr, D_rb, D_br, D_bb, in FP64 / FP32 / BF16, with ragged time chunks,
non-power-of-two volumes and several RHS counts."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import matfree

from gpu_support import Lattice, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-14, "fp32": 2e-6, "bf16": 1.5e-2}


def shapes(dims, nrhs, prec):
    V = int(np.prod(dims))
    out = []
    for sb in (64, 128, 256):
        for rg in sorted({1, nrhs}):
            for split in ((0, 1, 2) if prec == "bf16" else (0, 1)):
                for chunk in (0, 1, 8):
                    items = -(-V // sb) * -(-nrhs // rg)
                    grid = max(8, min(2048, -(-items // 8) * 8))
                    out.append(dict(SB=sb, RG=rg, split=split, grid=grid, chunk=chunk, march=0))
    v3 = dims[0] * dims[1] * dims[2]
    maxrg = 8 if prec == "fp64" else 12
    for T in sorted({1, 2, 3, 5, dims[3]}):
        if T > dims[3]:
            continue
        for rg in sorted({1, min(nrhs, maxrg)}):
            items = -(-v3 // 64) * -(-dims[3] // T) * -(-nrhs // rg)
            for chunk in (0, 1):
                grid = max(8, min(2048, -(-items // 8) * 8))
                out.append(dict(SB=64, RG=rg, split=0, grid=grid, chunk=chunk, march=T))
    return out


@pytest.mark.parametrize("dims,nrhs", [((8, 8, 8, 8), 3), ((4, 6, 8, 6), 1), ((8, 8, 8, 16), 12)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_block_apply_every_launch(dims, nrhs, prec):
    import torch

    lat = Lattice(dims, 0.5, 31)
    s = lat.schur(-0.25, "II", True, max_rhs=max(nrhs, 1))
    grg = lat.grg
    x = gaussian_vectors(12 * lat.V, nrhs, 31)
    xd = to_dev(x)
    out = torch.empty_like(xd)
    blocks = [(0, 0), (0, 1), (1, 0), (1, 1), (-1, -1)]
    want = {}
    for rows, cols in blocks:
        if rows < 0:
            want[(rows, cols)] = matfree.dirac_apply(lat.links, dims, -0.25, x)
        else:
            want[(rows, cols)] = matfree.block_apply(lat.links, dims, -0.25, s.q, s.nb, rows, cols, x)
    first = None
    for shp in shapes(dims, nrhs, prec):
        try:
            grg.grg_schur_set_launch(s.h, prec, nrhs, shp)
        except grg.GrgError:
            # only the shapes the library documents as invalid may be refused
            assert shp["march"] > 0 and 64 * shp["RG"] > (512 if prec == "fp64" else 768), shp
            continue
        for rows, cols in blocks:
            grg.grg_block_apply(s.h, prec, rows, cols, xd, out, nrhs)
            got = to_host(out)
            err = rel_err(got, want[(rows, cols)])
            assert err < TOL[prec], (shp, rows, cols, err)
            if (rows, cols) == (0, 0):
                if first is None:
                    first = got
                elif prec == "fp64":
                    # every shape evaluates the same sum up to its order
                    assert rel_err(got, first) < 1e-15
    s.close()
    lat.close()


def test_set_launch_rejects_bad_shapes():
    lat = Lattice((8, 8, 8, 8), 0.5, 1)
    s = lat.schur(-0.1, "I", False, max_rhs=12)
    grg = lat.grg
    bad = [dict(SB=96, RG=1, split=0, grid=64, chunk=0, march=0),
           dict(SB=64, RG=1, split=0, grid=60, chunk=0, march=0),
           dict(SB=64, RG=12, split=0, grid=64, chunk=0, march=9)]
    for b in bad:
        with pytest.raises(grg.GrgError):
            grg.grg_schur_set_launch(s.h, "bf16", 12, b)
    with pytest.raises(grg.GrgError):
        grg.grg_schur_set_launch(s.h, "fp64", 12, dict(SB=64, RG=12, split=0, grid=64, chunk=0, march=2))
    s.close()
    lat.close()


@pytest.mark.parametrize("rg", [4, 2, 1])
@pytest.mark.parametrize("inner", ["fp64", "bf16"])
def test_solver_with_march_kernel(inner, rg):
    """The solver's fused dot products with t-marching workgroups that hold
    all, half or one of the RHS (the per-RHS sums then come from several
    workgroups' items)."""
    lat = Lattice((8, 8, 8, 16), 0.5, 7)
    s = lat.schur(-0.3, "I", False, tol=1e-12, inner=inner, inner_tol=1e-2, max_rhs=4)
    xb = gaussian_vectors(12 * s.nb, 4, 7)
    y0, st0 = s.apply(xb)
    lat.grg.grg_schur_set_launch(s.h, inner, 4, dict(SB=64, RG=rg, split=0, grid=64, chunk=0, march=4))
    lat.grg.grg_schur_set_launch(s.h, "fp64", 4, dict(SB=64, RG=rg, split=0, grid=40, chunk=1, march=3))
    y1, st = s.apply(xb)
    assert st["converged"] and rel_err(y1, y0) < 1e-11
    # the same iterations: the dot products are the same sums
    assert abs(st["iters"] - st0["iters"]) <= 1
    s.close()
    lat.close()


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
def test_defect_correction_every_launch(inner):
    """The fused FP64 defect-correction step in every launch shape (site-
    parallel, and t-marching with all, some or one RHS per workgroup and
    ragged time chunks, for BF16 e also its LDS-ring form) gives the same
    solve."""
    lat = Lattice((8, 8, 8, 16), 0.5, 9)
    inner_tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}[inner]
    s = lat.schur(-0.3, "I", False, tol=1e-12, inner=inner, inner_tol=inner_tol, max_rhs=4)
    grg = lat.grg
    xb = gaussian_vectors(12 * s.nb, 4, 9)
    y0, st0 = s.apply(xb)
    assert st0["converged"]
    shapes = [dict(SB=sb, RG=1, split=0, grid=64, chunk=0, march=0) for sb in (64, 256)]
    for T in (1, 3, 16):
        for rg in (4, 2, 1):
            for chunk in (0, 1):
                shapes.append(dict(SB=64, RG=rg, split=0, grid=40, chunk=chunk, march=T))
                if inner == "bf16":  # the LDS-ring form (BF16 e only), also RHS group first
                    shapes.append(dict(SB=64, RG=rg, split=1, grid=40, chunk=chunk, march=T))
                    shapes.append(dict(SB=64, RG=rg, split=3, grid=40, chunk=chunk, march=T))
                    if chunk == 0 and rg < 4:  # whole z-planes of tiles per chunk
                        shapes.append(dict(SB=64, RG=rg, split=3, grid=16, chunk=8 * (4 // rg), march=T))
    for shp in shapes:
        grg.grg_schur_set_dc_launch(s.h, inner, 4, shp)
        assert grg.grg_schur_dc_launch_info(s.h, inner, 4)["march"] == shp["march"]
        y, st = s.apply(xb)
        assert st["converged"] and rel_err(y, y0) < 1e-11, (shp, st)
        assert abs(st["iters"] - st0["iters"]) <= 1 and st["outer"] == st0["outer"], (shp, st, st0)
    for bad in (dict(SB=96, RG=1, split=0, grid=64, chunk=0, march=0),
                dict(SB=64, RG=12, split=0, grid=64, chunk=0, march=2),
                dict(SB=64, RG=1, split=0, grid=60, chunk=0, march=2),
                dict(SB=64, RG=1, split=0, grid=64, chunk=0, march=17),
                dict(SB=64, RG=1, split=1, grid=64, chunk=0, march=0),
                dict(SB=64, RG=1, split=2, grid=64, chunk=0, march=2)):
        with pytest.raises(grg.GrgError):
            grg.grg_schur_set_dc_launch(s.h, inner, 4, bad)
    if inner != "bf16":
        for split in (1, 3):
            with pytest.raises(grg.GrgError):
                grg.grg_schur_set_dc_launch(s.h, inner, 4, dict(SB=64, RG=1, split=split, grid=64, chunk=0,
                                                                 march=2))
    s.close()
    lat.close()


def test_ring_defect_correction_needs_whole_x_rows_per_tile():
    """The LDS-ring form of the defect-correction step takes the x hops from
    the lanes of the same x-row: Lx must divide the 64 sites of a tile."""
    lat = Lattice((12, 4, 4, 8), 0.5, 10)  # 192 sites per slice, 64 % 12 != 0
    s = lat.schur(-0.3, "I", False, tol=1e-10, inner="bf16", inner_tol=1e-2, max_rhs=2)
    with pytest.raises(lat.grg.GrgError):
        lat.grg.grg_schur_set_dc_launch(s.h, "bf16", 2, dict(SB=64, RG=2, split=1, grid=8, chunk=0, march=2))
    # the t-marching form without the ring is fine there
    lat.grg.grg_schur_set_dc_launch(s.h, "bf16", 2, dict(SB=64, RG=2, split=0, grid=8, chunk=0, march=2))
    s.close()
    lat.close()
