"""The benchmark line's summary of the mixed-precision steps (host logic, no GPU)."""
import bench


def test_mixed_vs_plain_picks_the_fastest_reduced_precision_step():
    out = {
        "bdf2_step": {"order": 3, "fp64": {"ms": 120.0}, "fp32": {"ms": 90.0}, "bf16": {"ms": 80.0},
                      "gauss_seidel_fp64": {"ms": 60.0}, "gauss_seidel_bf16": {"ms": 70.0}},
        "batch": {"cases": 48, "bdf2_fp64": {"ms": 1600.0}, "bdf2_bf16": {"ms": 1000.0},
                  "gauss_seidel_fp64": {"ms": 700.0}, "gauss_seidel_bf16": {"ms": 800.0}},
    }
    mv = bench.mixed_vs_plain(out)
    # FP64 Gauss-Seidel is faster still, but it is not a reduced-precision step
    assert mv["bdf2_step"]["mixed"] == "gauss_seidel_bf16"
    assert mv["bdf2_step"]["ratio"] == 120.0 / 70.0
    assert mv["batch"]["mixed"] == "gauss_seidel_bf16" and mv["batch"]["plain_ms"] == 1600.0
    assert "bdf2_step_p4" not in mv


def test_mixed_vs_plain_without_steps():
    assert bench.mixed_vs_plain({"value": 1.0}) == {}
