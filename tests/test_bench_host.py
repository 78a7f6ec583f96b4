"""Host logic of bench.py (no GPU): the mapping from rocprofv3 kernel names to
the kernel names the library's profiler uses, which the traffic and roofline
figures are keyed by, and the multi-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("rocprof, key", [
    ("void dna::k_rgh_H<false, 0>(float const*, float const*)", "rgh_H"),
    ("dna::k_rgh_W<true, 2>(float const*)", "rgh_W"),
    ("dna::k_costf_H(float const*)", "costf_H"),
    ("dna::k_cand_H<2, 32>(float const*)", "cand_H"),
    ("dna::k_ratio<1, 0>(float const*)", "ratio_W"),
    ("dna::k_sp_grad<0, 1, false>(dna::SpV, float const*)", "sp_grad_H"),
    ("dna::k_sp_grad<1, 2, true>(dna::SpV, float const*)", "sp_grad_mu_W"),
    ("dna::k_sp_cost<0>(dna::SpV, float const*)", "sp_cost_H"),
    ("dna::k_sp_cost_comb<1>(dna::SpV, double const*)", "sp_cost_comb_W"),
    ("dna::k_sp_comb<1, true>(dna::SpV, float const*)", "sp_comb_W"),
    ("dna::k_sp_qz(dna::SpV, float const*)", "sp_qz"),
    ("void dna::k_hstep_cols<4, false, true>(dna::HColsArgs)", "hstep_cols"),
    ("dna::k_ratio<8>(dna::RatioArgs)", "ratio_H"),
    ("void dna::k_ratio<9, dna::Geo<64, 64, 16, 2, 2> >(dna::RatioKArgs)", "ratio_W"),
    ("_ZN3dna9k_ratio16IDF16bLi0ELb0ELi3EEEvNS_11Ratio16ArgsE", "ratio16_H"),
    ("_ZN3dna9k_ratio16IDF16_Li1ELb1ELi0EEEvNS_11Ratio16ArgsE", "qmax16"),
    ("_ZN3dna6k_gh16IDF16bLi0EEEvNS_5Ops16EllllPfS2_S2_NS_4FoldE", "gh16_H"),
    ("_ZN3dna8k_cost16IDF16_Li1ELb0EEEvPKfNS_5Ops16ElllPdPi", "cost16_W"),
    ("_ZN3dna8k_conv16IDF16bLb0EEEvNS_8ConvArgsE", "conv16"),
    ("void dna::k_gh2_W<dna::Geo<128, 64, 16, 2, 2> >(dna::Opnd, dna::Opnd)", "gh_W"),
    ("void dna::k_gh_H<dna::Geo<64, 128, 16, 2, 2>, dna::ProdGH3_H>(dna::Opnd)", "gh_H"),
])
def test_kernel_key(rocprof, key):
    assert bench.kernel_key(rocprof) == key


def test_hstep_cols_counts_both_passes():
    """The one-kernel H step does the gradient products and the two candidate
    reconstructions of a half-step: 8NRT algorithmic flops per launch."""
    assert bench.kernel_work("hstep_cols", 1024, 8192, 64) == ("flops", 8.0 * 1024 * 8192 * 64)
    assert bench.kernel_work("rgh_W", 1024, 8192, 64)[1] + bench.kernel_work("costf_W", 1024, 8192, 64)[1] == \
        bench.kernel_work("hstep_cols", 1024, 8192, 64)[1]


def test_traffic_missing_tag_is_none():
    assert bench.traffic_of("rgh_H", "no_such_workload") is None


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_strip_comments_keeps_code_and_literals():
    """The traffic files' source hash covers code only: comments and blank runs
    drop out, string and character literals (which may hold comment markers)
    stay."""
    src = ('int a = 1; // note "x"\n'
           '/* block\n comment */ int b = 2;\n\n'
           'const char* s = "not // a comment /* either */";\n'
           "char c = '\"'; char d = '\\\\';\n")
    out = bench.strip_comments(src)
    assert "note" not in out and "block" not in out
    assert '"not // a comment /* either */"' in out
    assert "int a = 1;" in out and "int b = 2;" in out and "char d = '\\\\';" in out
    assert bench.strip_comments(src.replace("note", "other note")) == out
