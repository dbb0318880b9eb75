"""Host-side logic of bench.py (no GPU): argument defaults, kernel-name
parsing, the algorithmic byte models behind the roofline figures, and the
rule that measured traffic is reported only for the kernel sources it was
measured on."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _parse(monkeypatch, *argv):
    monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
    return bench.parse()


def test_defaults_per_workload(monkeypatch):
    a = _parse(monkeypatch)
    assert (a.gpus, a.workload, a.n, a.steps, a.warmup) == (1, "c3", 512, 3, 1)
    assert (a.nu_pre, a.nu_post, a.warm_cycle) == (2, 3, "fmg")
    a = _parse(monkeypatch, "--workload", "c5")
    assert (a.n, a.steps, a.nu_pre, a.nu_post) == (768, 19, 2, 2)
    a = _parse(monkeypatch, "--workload", "c1", "--nu-pre", "1", "--nu-post", "1")
    assert (a.n, a.nu_pre, a.nu_post) == (64, 1, 1)


def test_split_name():
    assert bench.split_name("gs_fine_f32") == ("gs", 0)
    assert bench.split_name("resid_restrict_L3_f64") == ("resid_restrict", 3)
    assert bench.split_name("coarse_solve_coarsest_f32") == ("coarse_solve", -1)
    assert bench.split_name("op_multidot_zf32") == ("op_multidot_zf32", None)


@pytest.mark.parametrize("s", [4, 8])
def test_byte_models(s):
    """Bytes per cell written out from what each kernel reads and writes
    (the finest level colour-split: one colour is half a field)."""
    b = bench.bytes_per_cell
    assert b("sym", 0, s) == 3.5 * s            # old X half, a, B read; X written
    assert b("gs", 0, s) == 2.5 * s
    assert b("sym_first", 0, s) == 8 + 3 * s
    assert b("resid_restrict", 0, s) == 3 * s + s / 8
    assert b("gs", 2, s) == 5 * s               # x, 3 faces, b and x of one colour
    assert b("prolong_add", 0, s, nu_post=0) == 2 * s + s / 8
    c = bench.cheb_bytes_per_cell
    assert c("cheb_resid", 0, s) == 2 * s + 16
    assert c("cheb_resid", 1, s) == 6 * s
    assert c("cheb_update", 0, s) == (3 * s + 5 * s + 4 * s + 5 * s) / 4
    assert c("ssor", 3, s) == b("gs", 3, s) and c("ssor_first", 3, s) == b("gs_first", 3, s)
    assert bench.outer_bytes("op_multidot_zf32", 3, s) == s + 8 + 8 + 3 * 8  # z, a read, w written, 3 vectors


def test_nv_sequence_restarts():
    assert bench.nv_sequence(5, 10) == [1, 2, 3, 4, 5]
    assert bench.nv_sequence(12, 5) == [1, 2, 3, 4, 5, 1, 2, 3, 4, 5, 1, 2]


def test_traffic_only_for_matching_sources(monkeypatch, tmp_path):
    f = tmp_path / "traffic.md"
    f.write_text("traffic_bytes_per_launch: 2141258775\nkernel_source_sha256_16: 0123456789abcdef\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    assert bench.measured_traffic() == 2141258775.0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "fedcba9876543210")
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
