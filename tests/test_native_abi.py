"""CPU-side checks of the C ABI: libns.so loads and exports every entry
point that include/ns.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ns.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(ns_[A-Za-z0-9_]+)\s*\(", src))
    return sorted(n for n in names if n not in ("ns_ctx",))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ns_init", "ns_step_batch", "ns_logZ", "ns_run", "ns_get_dead", "ns_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2608_28514_amd import native
    lib = ctypes.CDLL(native.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\sT\s(ns_[A-Za-z0-9_]+)", out))
    assert set(_declared()) <= exported


def test_binding_signatures_load_and_defaults():
    from paper_2608_28514_amd import native
    c = native.ns_config_default()
    assert c.slice_steps_per_dim == 5 and c.hist_cap == 32 and c.correction == 3
    assert abs(c.stop_frac - 1e-3) < 1e-18


def test_invalid_arguments_are_rejected_without_a_device():
    from paper_2608_28514_amd import native, workloads
    spec = workloads.likelihood(1)
    c = native.ns_config_default()
    import pytest
    with pytest.raises(native.NsError, match="NS_EINVAL"):
        native.ns_init(spec, 1, c, stream=0)         # N < 2
    bad = dict(spec, d=33, lo=[0.0] * 33, hi=[1.0] * 33)
    with pytest.raises(native.NsError, match="NS_EINVAL"):
        native.ns_init(bad, 100, c, stream=0)
    bad = dict(spec, hi=spec["lo"])
    with pytest.raises(native.NsError, match="NS_EINVAL"):
        native.ns_init(bad, 100, c, stream=0)


def test_oracle_and_library_share_no_code():
    """The oracle neither includes the library's headers nor imports its
    package, and the library never includes or imports the oracle."""
    orc = os.path.join(ROOT, "oracle")
    lib = os.path.join(ROOT, "paper_2608_28514_amd")
    for f in os.listdir(orc):
        if f.endswith((".c", ".h", ".py")):
            s = open(os.path.join(orc, f)).read()
            assert not re.search(r"^\s*(import|from)\s+paper_2608_28514_amd", s, re.M), f
            assert not re.search(r'#include\s+".*(ns\.h|ns_device|ns_internal)', s), f
    for root, _, files in os.walk(lib):
        for f in files:
            if f.endswith((".hip", ".hpp", ".py", ".h")):
                s = open(os.path.join(root, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", s, re.M), f
                assert "ns_oracle" not in s, f
