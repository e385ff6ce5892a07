"""Host logic of the profile summaries that bench.py reads: kernel names map
to the families turpy_profile uses, and committed counter figures are used
only for the library sources they were taken on."""
import json

from paper_2604_07248_amd import prof_summary as ps


def test_kernel_families():
    ns = "void turpy::(anonymous namespace)::"
    cases = {
        "row_relay_kernel<1024>(turpy::RowArgs)": "row_fwd",
        "row_pair_kernel<1024, 1, false>(turpy::RowArgs)": "row_fwd",
        "row_pair_kernel<1024, 1, true>(turpy::RowArgs)": "row_bwd",
        "row_pass_kernel<1024, 0, false>(turpy::RowArgs)": "row_plain",
        "row_pass_kernel<16, 2, true>(turpy::RowArgs)": "row_bwd",
        "col_pass_kernel<1024, 0, 8>(turpy::ColArgs)": "col",
        "synth_col_kernel<1024, 4>(turpy::SynthArgs)": "synth",
        "stats_kernel(turpy::StatsArgs)": "stats",
        "copy_kernel(HIP_vector_type<float, 2u> const*, long, HIP_vector_type<float, 2u>*, long, long)": "copy",
    }
    for name, fam in cases.items():
        assert ps.family(ns + name) == fam, name
    # runtime and PyTorch kernels belong to no family
    assert ps.family("__amd_rocclr_copyBuffer") is None
    assert ps.family("void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>>") is None


def test_traffic_only_for_matching_sources(tmp_path):
    fams = {"row_fwd": {"read_bytes": 1, "write_bytes": 2, "bytes_per_launch": 3}}

    def write(sha):
        doc = {"traffic": {"leg": "fwd", "sources_sha256": sha, "families": fams}}
        (tmp_path / "fwd_x_hbm_traffic.md").write_text("# t\n\n```json\n" + json.dumps(doc) + "\n```\n")

    write(ps.sources_sha256())
    assert ps.load_traffic(str(tmp_path), "fwd") == {"row_fwd": 3}
    write("0" * 64)
    assert ps.load_traffic(str(tmp_path), "fwd") == {}

