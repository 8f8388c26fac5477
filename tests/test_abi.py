"""The C-ABI library loads and exports every entry point include/aenet_gpu.h
declares; the Python binding names the same set.  No compute call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aenet_gpu.h")
LIB = os.path.join(ROOT, "paper_2107_11311_amd", "libaenet_gpu.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aenet_[a-z_]+)\s*\(", text)))


def test_header_declares_the_calls():
    names = declared()
    for n in ("aenet_setup", "aenet_energy_forces", "aenet_md_step", "aenet_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2107_11311_amd import aenet
    assert sorted(aenet.EXPORTS) == declared()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2107_11311_amd import aenet
    with pytest.raises(RuntimeError):
        aenet.load(str(tmp_path / "missing.so"))


PROBE_LIB = os.path.join(ROOT, "paper_2107_11311_amd", "libaenet_probe.so")


@pytest.mark.skipif(not os.path.exists(PROBE_LIB), reason="probe library not built")
def test_peak_probes_export_what_the_benchmark_calls():
    """bench.py's arithmetic peak microbenchmarks (a separate library; no part
    of the method) export every probe the benchmark names."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    lib = ctypes.CDLL(PROBE_LIB)
    for fn, _, published in bench.PEAK_PROBES.values():
        assert hasattr(lib, fn), fn
        assert published > 0
    # the probe library is not part of the C ABI
    assert not any(n.startswith("probe_") for n in declared())
