"""Host logic of bench.py that needs no GPU: the refusal of more than one GPU,
the algorithmic byte model behind the roofline figures (against the
per-pixel figures of the fused design's byte count and against the HBM
traffic the committed counter summaries measured), and the roofline entry."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2604_07248_amd import prof_summary, workloads  # noqa: E402


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr


def _per_pixel(w, leg):
    p = w.path
    return sum(bench.step_bytes(p, leg).values()) / (p.realizations * p.num_screens * p.n * p.n)


@pytest.mark.parametrize("leg,w,expected", [("fwd", workloads.headline(), 40.0),
                                            ("fwdbwd", workloads.headline(), 100.0),
                                            ("ar", workloads.config3(), 48.0)])
def test_bytes_per_screen_step_and_pixel(leg, w, expected):
    """Per realization, screen-step and pixel the fused design moves about
    40 bytes forward (two passes reading and writing 8 bytes, the screen's
    half scratch plane written and read), 100 with checkpoints and the adjoint,
    48 with the AR state read and written; the one-off planes (source, final
    pass, moments) add the rest."""
    b = _per_pixel(w, leg)
    assert expected <= b <= 1.03 * expected, b


def test_headline_bytes_pinned():
    fams = bench.step_bytes(workloads.headline().path, "fwd")
    assert sum(fams.values()) == 22_087_204_864
    assert fams["row_fwd"] // 8 == 1_276_116_992  # per launch, the roofline's figure
    assert fams["col"] == (2 + 2 * 64 * 8) * 1024 * 1024 * 8


# launches per step of each family (headline workload, M = 8)
LAUNCHES = {"fwd": {"col": 9, "row_fwd": 8, "synth": 8, "row_moments": 1, "row_plain": 1},
            "fwdbwd": {"col": 18, "row_fwd": 8, "row_bwd": 8, "synth": 8, "row_plain": 4, "sum": 1}}


@pytest.mark.parametrize("leg", ["fwd", "fwdbwd"])
def test_measured_traffic_equals_the_byte_model(leg):
    """The committed FETCH_SIZE + WRITE_SIZE summaries (when taken on the
    current sources) equal the algorithmic bytes per launch within 2 %: no
    kernel re-reads."""
    measured = prof_summary.load_traffic(os.path.join(ROOT, "profiles"), leg)
    if not measured:
        pytest.skip("the committed counter summary was taken on other library sources")
    fams = bench.step_bytes(workloads.headline().path, leg)
    for fam, n in LAUNCHES[leg].items():
        algo = fams[fam] / n
        assert abs(measured[fam] - algo) <= 0.02 * algo, (fam, measured[fam], algo)


def test_roofline_entry():
    path = workloads.headline().path
    table = {"row_fwd": {"bytes_per_launch": 1.0e9, "avg_us": 250.0, "timed_region_avg_us": 200.0}}
    r = bench.roofline(table, "row_fwd", {"row_fwd": 1.01e9}, path, "fwd", 4.0e-3)
    assert r["achieved"] == pytest.approx(5000.0) and r["frac"] == pytest.approx(0.625)
    assert r["traffic"] == 1.01e9 and r["peak"] == 8000.0
    assert r["step"]["achieved"] == pytest.approx(22_087_204_864 / 4.0e-3 / 1e9)
