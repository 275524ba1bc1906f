"""The C-ABI library builds, loads and exports every symbol include/grg.h
declares; host-only logic (the permutation builder, parameter defaults) is
checked without a GPU."""
import os
import re

import numpy as np
import pytest

import paper_0704_2341_amd as grg
from paper_0704_2341_amd import binding
from oracle import dense

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "grg.h")) as f:
        text = f.read()
    return set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(grg_\w+)\s*\(", text, re.M))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_0704_2341_amd import build

        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    syms = header_symbols()
    assert len(syms) >= 15
    assert syms == set(binding.EXPORTS)
    for s in syms:
        assert hasattr(lib, s), s


def test_library_is_gfx950_hip(lib):
    assert "gfx950" in grg.grg_version()


def test_params_default():
    p = grg.grg_solver_params_default()
    assert p.tol == 1e-10 and p.restart >= 1 and p.max_rhs == 12 and p.inner == grg.GRG_FP64


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 2), (8, 8, 8, 16)])
@pytest.mark.parametrize("kind,inv", [("I", False), ("II", False), ("I", True), ("II", True)])
def test_permutation_matches_oracle(dims, kind, inv):
    q, nb = grg.grg_permutation_block(dims, 1 if kind == "I" else 2, inv)
    qo, nbo = dense.permutation_block(dims, kind, inv)
    assert nb == nbo
    assert np.array_equal(q, qo)


def test_permutation_rejects_odd_extent():
    with pytest.raises(grg.GrgError) as e:
        grg.grg_permutation_block((4, 4, 4, 5), 1)
    assert e.value.status == grg.GRG_EODD_EXTENT
    with pytest.raises(grg.GrgError) as e:
        grg.grg_permutation_block((4, 4, 4, 4), 3)
    assert e.value.status == grg.GRG_EINVAL
