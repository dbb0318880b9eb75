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


@pytest.mark.parametrize("kernel", ["sym_fine_f32", "sym_fine_f64"])
def test_traffic_only_for_matching_sources(monkeypatch, tmp_path, kernel):
    f = tmp_path / "traffic.md"
    f.write_text("traffic_bytes_per_launch: 2141258775\nkernel_source_sha256_16: 0123456789abcdef\n")
    monkeypatch.setitem(bench.TRAFFIC_FILES, kernel, str(f))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "0123456789abcdef")
    assert bench.measured_traffic(kernel) == 2141258775.0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k: "fedcba9876543210")
    assert bench.measured_traffic(kernel) is None
    monkeypatch.setitem(bench.TRAFFIC_FILES, kernel, str(tmp_path / "missing.md"))
    assert bench.measured_traffic(kernel) is None
    assert bench.measured_traffic("resid_restrict_fine_f32") is None


def test_kernel_sources_hash_per_kernel():
    """Each counted kernel hashes the device sources plus its own launch
    function (the float32 and float64 fused sweeps share one)."""
    h32, h64 = bench.kernel_source_hash("sym_fine_f32"), bench.kernel_source_hash("sym_fine_f64")
    assert len(h32) == 16 and h32 == h64


def test_hashed_sources_close_over_the_fused_sweep():
    """The hash covers everything the fused sweep's device code is compiled
    from: its header includes only the shared helpers, which include only
    system headers, so a change to any other kernel keeps the counted
    traffic valid and a change to these files drops it."""
    import re
    csrc = os.path.join(os.path.dirname(bench.__file__), "paper_1812_08606_amd", "csrc")
    for kernel in ("sym_fine_f32", "sym_fine_f64"):
        files = bench.KERNEL_SOURCES[kernel]
        for f in files:
            text = open(os.path.join(csrc, f)).read()
            for inc in re.findall(r'#include\s+"([^"]+)"', text):
                assert inc in files, (f, inc)
        assert "void k_sym_split(" in open(os.path.join(csrc, "gmg_sym.hpp")).read()


def test_kernel_table_and_roofline():
    """Byte models per kernel from an event pass: the fused sweep's 14 B/cell
    per launch at 512^3 (mixed) over its average launch, and the float64
    half-sweep's 20 B/cell."""
    N = 512 ** 3
    prof = {"sym_fine_f32": (6.9, 10), "op_multidot_zf32": (1.0, 5), "gs_fine_f64": (3.6, 5)}
    table, total = bench.kernel_table(prof, 1, [5], 4, N)
    roof = bench.roofline_of(table, 100.0, False)
    assert roof["kernel"] == "sym_fine_f32" and roof["bytes_per_launch"] == 14 * N
    assert abs(roof["achieved"] - 14 * N / 0.69e-3 / 1e9) < 0.1 and roof["traffic"] is None
    table64, _ = bench.kernel_table({"gs_fine_f64": (3.6, 5)}, 1, [5], 8, N)
    assert bench.roofline_of(table64, 100.0, False)["bytes_per_launch"] == 20 * N
    assert total > 0


def test_more_than_one_gpu_is_refused(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2


def test_coarse_fused_sweep_byte_model():
    """The coarse levels' fused sweep moves 5.5 s per cell (old second colour
    s/2, three face arrays, b read; x written), against 2 x 5 s for the two
    half-sweeps it replaces; its rows get a bandwidth in the kernel table."""
    assert bench.bytes_per_cell("sym", 1, 4) == 22 and bench.bytes_per_cell("sym", 2, 8) == 44
    assert bench.bytes_per_cell("sym_first", 1, 4) == 20
    assert bench.bytes_per_cell("gs", 1, 4) == 20
    N = 512 ** 3
    table, _ = bench.kernel_table({"sym_L1_f32": (6.7, 45)}, 1, [5], 4, N)
    row = table[0]
    assert row[0] == "sym_L1_f32" and row[5] == 22 * (N // 8)


def test_fused_residual_sweep_byte_model():
    """The finest level's last pre-smoothing sweep, fused with the residual
    restriction, moves the sweep's 3.5 s per cell plus the coarse right side
    (s / 8), in place of the sweep and a 3 s + s / 8 residual pass."""
    assert bench.bytes_per_cell("sym_resid", 0, 4) == 14.5 and bench.bytes_per_cell("sym_resid", 0, 8) == 29
    assert bench.bytes_per_cell("sym", 0, 4) + bench.bytes_per_cell("resid_restrict", 0, 4) == 26.5
    N = 512 ** 3
    table, _ = bench.kernel_table({"sym_resid_fine_f32": (2.6, 5)}, 1, [5], 4, N)
    assert table[0][0] == "sym_resid_fine_f32" and table[0][5] == 14.5 * N
