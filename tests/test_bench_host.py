"""Host logic of the benchmark (CPU): the committed HBM byte counters are used for
`roofline.traffic` only while the kernels' code is the code they were taken on."""
import os
import re
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A copy of the kernels source and of the counters summary under a scratch root."""
    (tmp_path / "paper_2604_07170_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = os.path.join("paper_2604_07170_amd", "csrc", "wfp2d_kernels.hip")
    shutil.copy(os.path.join(ROOT, src), tmp_path / src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the copied summaries are marked as taken on the copied source, whatever the committed state
    for form in ("mixed", "fp64"):
        prof = os.path.join("profiles", f"hbm_counters_cfg4_M1e6_{form}.md")
        text = re.sub(r"code sha256 prefix: [0-9a-f]{16}", "code sha256 prefix: " + bench.kernels_digest(),
                      open(os.path.join(ROOT, prof)).read())
        (tmp_path / prof).write_text(text)
    return tmp_path / src


def test_lookup_by_kernel_name(tree):
    assert bench.measured_traffic("k_near") is not None
    assert bench.measured_traffic("k_no_such_kernel") is None


def test_comment_edits_keep_and_code_edits_drop_the_counters(tree):
    base = bench.kernels_digest()
    bytes0 = bench.measured_traffic("k_local_pc")
    assert bytes0 is not None and bytes0 > 1e9
    text = tree.read_text()
    tree.write_text("// a new comment line\n\n" + text.replace("{\n", "{  /* note */\n", 1))
    assert bench.kernels_digest() == base
    assert bench.measured_traffic("k_local_pc") == bytes0
    tree.write_text(text + "\nstatic int wfp2d_changed_code = 1;\n")
    assert bench.kernels_digest() != base
    assert bench.measured_traffic("k_local_pc") is None


def test_missing_summary_gives_no_traffic(tree):
    os.remove(tree.parents[2] / "profiles" / "hbm_counters_cfg4_M1e6_mixed.md")
    assert bench.measured_traffic("k_local_pc") is None


def test_lookup_is_keyed_by_precision_and_template(tree):
    assert bench.measured_traffic("k_near", ("float",), "mixed") is not None
    assert bench.measured_traffic("k_near", ("double",), "mixed") is None      # an FP64 kernel: not profiled
    assert bench.measured_traffic("k_near", ("float",), "fp64") is None        # the FP64 summary lists k_near<double>
    assert bench.measured_traffic("k_near", ("double",), "fp64") is not None
    assert bench.measured_traffic("k_local_pc", (35, 16), "mixed") is not None
    assert bench.measured_traffic("k_local_pc", (35, 20), "mixed") is None
    # several instantiations match a bare base name: ambiguous, so no figure
    assert bench.measured_traffic("k_fft_t1", (), "mixed") is None
    assert bench.measured_traffic("k_fft_t1", ("float", 1), "mixed") is not None


def test_kernel_row_names():
    assert bench.kernel_row_matches("wfp2d::k_local_pc<35, 16, 4>", "k_local_pc", (35, 16))
    assert not bench.kernel_row_matches("wfp2d::k_local_pc<35, 16, 4>", "k_local", ())
    assert bench.kernel_row_matches("wfp2d::k_combine", "k_combine", ())
    assert not bench.kernel_row_matches("wfp2d::k_combine_dot", "k_combine", ())


def test_timed_window_ends_at_the_last_step_after_far_onset():
    # 10^6-source workload: nt = 6000, LA = 4300, W = 16
    assert bench.timed_window(6000, 4300, 16, 200) == (5801, 6000)
    assert bench.timed_window(6000, 4300, 16, 20) == (5981, 6000)
    first, last = bench.timed_window(6000, 4300, 16, 3000)
    assert first > 4300 + 16 and last - first + 1 == 3000
