"""Host-side logic of the benchmark (no GPU): the one-GPU guard, the
algorithmic byte counts the roofline divides by, the profiler names of the
dominant launch, and the traffic table's lookup by launch shape and source
fingerprint."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr


def test_algorithmic_bytes():
    b = _bench()
    V = 32 ** 4
    # full stencil, BF16, 12 RHS: in + out per RHS (2 x 12 complex of 4 bytes)
    # and 4 links of 9 complex per site
    assert b.dslash_bytes_per_launch("bf16", V, 12) == V * (12 * 2 * 12 * 4 + 4 * 9 * 4)
    # reduced operator, averaged over its halves: (V + 1.5 V) spinor fields
    # per RHS and all sites' 4 links per half
    assert b.eo_bytes_per_launch("bf16", V, 12, 20, 5) == 905_969_664
    assert b.eo_bytes_per_launch("fp64", V, 1, 20, 5) == V * ((1 + 1.5) / 2 * 12 * 16 + 4 * 9 * 16)


@pytest.mark.parametrize("split,rg,sym", [(7, 1, "eo_plane_kernel<0, 0, 1> + eo_plane_kernel<0, 2, 1>"),
                                          (7, 2, "eo_plane_kernel<0, 0, 2> + eo_plane_kernel<0, 2, 2>"),
                                          (3, 3, "eo_hop_kernel<2, 3, 0>"), (1, 3, "eo_hop_kernel<2, 1, 0>")])
def test_dominant_launch_names(split, rg, sym):
    """The kernel names the profiler reports (template arguments as the
    demangler prints them: the plane form's planes per workgroup are its RG)."""
    b = _bench()
    info = dict(SB=512 if split == 7 else 256, RG=rg, split=split, grid=3072, chunk=0,
                march=4 if split in (3, 7) else 0)
    d = b.launch_descriptor(info, "bf16", 40, eo=True)
    assert d["symbol"] == sym
    assert d["grid_size"] == info["grid"] * info["SB"]
    assert d["shape"] == info


@pytest.mark.parametrize("prec,info,sym,gs", [
    ("fp64", dict(SB=64, RG=6, split=0, grid=2048, chunk=0, march=16), "march_kernel<grg::StoreEpi<0> >", 2048 * 64 * 6),
    ("bf16", dict(SB=256, RG=3, split=2, grid=4096, chunk=0, march=0), "dslash_kernel<2, 2>", 4096 * 256),
    ("fp32", dict(SB=64, RG=1, split=1, grid=2048, chunk=64, march=0), "dslash_kernel<1, 1>", 2048 * 64)])
def test_full_stencil_launch_names(prec, info, sym, gs):
    b = _bench()
    d = b.launch_descriptor(info, prec, 10)
    assert d["symbol"] == sym and d["grid_size"] == gs


def test_stencil_launch_pins_parse():
    b = _bench()
    got = b.parse_stencil_launches("fp64_nrhs1=128,1,0,512,1,0; bf16_nrhs12=256,3,2,4096,0,0;")
    assert got == {"fp64_nrhs1": [128, 1, 0, 512, 1, 0], "bf16_nrhs12": [256, 3, 2, 4096, 0, 0]}


def test_traffic_lookup_by_shape_and_sources(tmp_path):
    from paper_0704_2341_amd import profiling as P

    shape = dict(SB=512, RG=1, split=7, grid=3072, chunk=0, march=4)
    key = P.traffic_key("bf16_eo", 12, (32, 32, 32, 32), shape)
    assert key.endswith("SB512_RG1_split7_grid3072_chunk0_march4")
    other = P.traffic_key("bf16_eo", 12, (32, 32, 32, 32), dict(shape, march=8))
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps({"kernel_source_sha256": P.kernel_source_hash(),
                                "kernels": {key: {"hbm_bytes_per_launch": 1.5e9}}}))
    assert P.measured_traffic(key, str(path)) == 1.5e9
    assert P.measured_traffic(other, str(path)) is None  # no counters for that shape
    path.write_text(json.dumps({"kernel_source_sha256": "0" * 64,
                                "kernels": {key: {"hbm_bytes_per_launch": 1.5e9}}}))
    assert P.measured_traffic(key, str(path)) is None  # taken on other sources
    assert P.measured_traffic(key, str(tmp_path / "missing.json")) is None
