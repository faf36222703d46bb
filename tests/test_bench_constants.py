"""bench.py's algorithmic constants agree with what they are derived from."""
import bench
from oracle import oracle as orc
from paper_2503_04558_amd import workload as wl


def test_flop_count_matches_oracle_count():
    """FP64_OPS_PER_PARTICLE_STEP is the oracle's operation count (counting
    scalar type) per particle-step on the benchmark workload."""
    g = wl.make_grid(2048, 2048, 0.99)
    parts = wl.pairs(g, 500, kind="mj", seed=0, params=dict(T=0.1, vphi=0.1))
    ops = orc.count_ops(g, wl.species_table(), parts, wl.wald_fields(g), wl.crossing_dt(g))
    assert ops["particles"] == 1000
    assert abs(ops["total"] - bench.FP64_OPS_PER_PARTICLE_STEP) < 1.0, ops


def test_particle_bytes():
    # cell int32, six float64 arrays and a uint8 species read; cell and five float64 written
    assert bench.FP64_PARTICLE_BYTES == (4 + 6 * 8 + 1) + (4 + 5 * 8)


def test_traffic_figure_tracks_kernel_sources(tmp_path, monkeypatch):
    """bench.py reports the measured HBM traffic only for the kernel sources
    it was measured on."""
    import bench

    t = bench.measured_traffic()
    if t:
        assert {"f64", "split"} <= set(t) and all(v > 1e9 for v in t.values())
    stale = tmp_path / "p.md"
    stale.write_text("traffic_bytes_per_launch f64=1e10 split=5e9 sources=0000\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench.measured_traffic() == {}


def test_field_traffic_figure_tracks_field_sources(tmp_path):
    """The field leg's measured traffic is keyed to the field kernel sources
    and is within a few percent above the algorithmic bytes of a step."""
    import bench

    t = bench.measured_traffic(bench.FIELD_TRAFFIC_PROFILE, bench.FIELD_SOURCES)
    if t:
        plane = 2049 * 2049 * 8
        alg = plane * (bench.FIELD_PLANES_PREDICTOR + 7 * bench.FIELD_PLANES_CORRECTOR)
        assert 1.0 <= t["step"] / alg < 1.2
        assert abs(t["predictor"] + 7 * t["corrector"] - t["step"]) < 1e-3 * t["step"]
    stale = tmp_path / "f.md"
    stale.write_text("traffic_bytes_per_launch step=1e9 sources=0000\n")
    assert bench.measured_traffic(str(stale), bench.FIELD_SOURCES) == {}
