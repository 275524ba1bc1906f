"""BF16 stencils entry by entry against the oracle evaluated exactly on the
values the kernels read.

A BF16 evaluation reads its inputs and links as bfloat16 values (reached
from FP64 through FP32), forms every product exactly in FP32 and sums in
FP32, and stores its output once in bfloat16.  So the oracle is run on the
same bfloat16 input and link values, and the only differences left are the
FP32 sums and the output's rounding:

    |y - y_r| <= u |y_r| + 2^-16 sum|terms|        (u = 2^-8),

with sum|terms| the oracle's sum of the absolute values of the products.
The reduced operator stores its intermediate field H_qp x_p in bfloat16 too,
which adds u (|H_pq| |t_r|) / |d| with t_r the exact intermediate.  A wrong
operand in a single hop of a single entry (a stale register, a wrong
neighbour, a missed sign) moves that entry by about one product, far above
these bounds; a per-RHS norm at a percent would not see it.  Every launch
form of the full stencil and of the half-lattice stencils is checked, at 8^4
and at an asymmetric shape with ragged tiles."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import matfree, rounding

from gpu_support import Lattice, to_dev, to_host
from test_gpu_eo import RA_LAUNCHES
from test_gpu_kernels import shapes

pytestmark = pytest.mark.gpu

U = rounding.UNIT_ROUNDOFF["bf16"]
SHAPES = [(8, 8, 8, 8), (16, 8, 4, 6)]


def _bound_ok(y, yr, extra):
    bound = U * (1 + 2 ** -7) * np.abs(yr) + extra
    ratio = np.abs(y - yr) / np.maximum(bound, 1e-300)
    return bool(np.all(np.abs(y - yr) <= bound)), float(ratio.max())


@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_full_stencil_every_launch(dims):
    import torch

    nrhs, m0 = 3, -0.3
    lat = Lattice(dims, 0.5, 61)
    s = lat.schur(m0, "II", True, max_rhs=nrhs)
    grg = lat.grg
    x = gaussian_vectors(12 * lat.V, nrhs, 61)
    lr, xr = rounding.bf16_value(lat.links), rounding.bf16_value(x)
    want, extra = {}, {}
    for rows, cols in ((0, 0), (-1, -1)):
        if rows < 0:
            want[rows] = matfree.dirac_apply(lr, dims, m0, xr)
            # no coarse sites (n_coarse 0): rows and columns over every site
            terms = matfree.block_apply_abs(lr, dims, m0, np.arange(lat.V), 0, 0, 0, xr)
        else:
            want[rows] = matfree.block_apply(lr, dims, m0, s.q, s.nb, rows, cols, xr)
            terms = matfree.block_apply_abs(lr, dims, m0, s.q, s.nb, rows, cols, xr)
        extra[rows] = 2.0 ** -16 * terms
    xd = to_dev(x)
    out = torch.empty_like(xd)
    n = 0
    for shp in shapes(dims, nrhs, "bf16"):
        try:
            grg.grg_schur_set_launch(s.h, "bf16", nrhs, shp)
        except grg.GrgError:
            assert shp["march"] > 0, shp
            continue
        for rows, cols in ((0, 0), (-1, -1)):
            grg.grg_block_apply(s.h, "bf16", rows, cols, xd, out, nrhs)
            ok, worst = _bound_ok(to_host(out), want[rows], extra[rows])
            assert ok, (shp, rows, worst)
        n += 1
    print(f"{dims}: {n} launch shapes entry-wise within the bound", flush=True)
    assert n > 10
    s.close()
    lat.close()


@pytest.mark.parametrize("dims", SHAPES + [(16, 8, 16, 4)], ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("kind,inv", [("I", False), ("II", True)])
def test_half_stencil_every_form(dims, kind, inv):
    import torch

    nrhs, m0 = 5, -0.3
    lat = Lattice(dims, 0.5, 62)
    s = lat.schur(m0, kind, inv, tol=1e-10, inner="bf16", max_rhs=nrhs)
    grg = lat.grg
    x = gaussian_vectors(12 * lat.V, nrhs, 62)
    lr, xr = rounding.bf16_value(lat.links), rounding.bf16_value(x)
    par = matfree.site_parity(dims)
    d = abs(4 + m0)
    want, extra = {}, {}
    for p in (0, 1):
        want[p] = matfree.reduced_apply(lr, dims, m0, s.q, s.nb, p, xr)
        t = matfree.reduced_intermediate(lr, dims, m0, s.q, s.nb, p, xr)
        ht = matfree.block_apply_abs(lr, dims, m0, s.q, s.nb, 0, 0, np.abs(t).astype(complex), diag=False)
        ht = (ht.reshape(nrhs, lat.V, 12) * (par == p)[None, :, None]).reshape(nrhs, -1)
        terms = matfree.reduced_apply_abs(lr, dims, m0, s.q, s.nb, p, xr)
        extra[p] = U * (1 + 2 ** -7) * ht / d + 2.0 ** -16 * terms
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    plane = dims[0] // 2 * dims[1]
    n = 0
    forms = dict(RA_LAUNCHES)
    forms["plane-two-planes"] = (64, 2, 7, 16, 0, 2)
    for form, launch in forms.items():
        try:
            grg.grg_schur_set_launch(s.h, "bf16", nrhs, launch, eo=True)
        except grg.GrgError:
            # refused only where documented: a plane form whose workgroup is
            # not this lattice's x-y plane, a marching form longer than Lt
            assert (launch[2] == 7 and launch[0] != plane) or (launch[2] in (3, 7) and launch[5] > dims[3]) \
                or (launch[2] == 7 and launch[1] == 2 and dims[2] % 16), (form, dims)
            continue
        for p in (0, 1):
            grg.grg_reduced_apply(s.h, "bf16", p, xd, yd, nrhs)
            ok, worst = _bound_ok(to_host(yd), want[p], extra[p])
            print(f"{dims} {kind}{'-inv' if inv else ''} {form} parity {p}: worst/bound {worst:.3f}",
                  flush=True)
            assert ok, (form, p, worst)
        n += 1
    assert n >= len(forms) - 4
    s.close()
    lat.close()
