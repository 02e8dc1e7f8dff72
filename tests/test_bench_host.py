"""Host logic of bench.py and the entry module, without a GPU: the
algorithmic byte count of the measured stack, the rule that counter
traffic is reported only for the kernel sources it was taken on, and the
one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_measured_stack():
    # read the uint16 stack once, write the FP32 volume and two projections:
    # 2NRC + 4NRW + 8RW on 512 x 512 x 2048, W = 3504
    assert bench.algorithmic_bytes(512, 512, 2048, 3504) == 4_762_304_512
    assert bench.algorithmic_bytes(1, 1, 1, 1) == 2 + 4 + 8


def _summary(path, digest, nbytes):
    path.write_text("# counters\n\n"
                    f"- kernel_sources_sha256_16: {digest}\n"
                    f"- hbm_bytes_per_launch: {nbytes}\n")


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    p = tmp_path / "pmc.md"
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(p))
    assert bench.measured_traffic() is None              # no summary
    _summary(p, bench.kernel_hash(), 4_800_000_000)
    assert bench.measured_traffic() == 4_800_000_000
    _summary(p, "0" * 16, 4_800_000_000)                 # other sources
    assert bench.measured_traffic() is None


def test_kernel_hash_follows_the_kernel_sources(tmp_path, monkeypatch):
    h0 = bench.kernel_hash()
    src = tmp_path / "k.hpp"
    src.write_text("a")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    monkeypatch.setattr(bench, "ROOT", "/")
    h1 = bench.kernel_hash()
    src.write_text("b")
    assert bench.kernel_hash() != h1 and h1 != h0


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_entry_module_has_build_and_smoke():
    sys.path.insert(0, ROOT)
    import __graft_entry__ as g
    assert callable(g.build) and callable(g.smoke)


def test_extras_keys_never_shadow_the_line_contract():
    """Every extra measurement lands under its own key; none may replace a
    field the one-line contract defines (metric, value, scaling, ...)."""
    import re
    src = open(os.path.join(ROOT, "bench.py")).read()
    extra_keys = set(re.findall(r'ext\["(\w+)"\]\s*=', src))
    contract = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"}
    assert extra_keys and not extra_keys & contract, extra_keys & contract
