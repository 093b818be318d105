"""Host logic of bench.py's roofline.traffic: the committed HBM counter summary
is used only for the workload, kernel sources, product engine and tile layout it
was taken on."""
import bench


def summary(tmp_path, workload="ea32", engine="valu", layout="compact", sha=None, value="2159731206"):
    sha = bench.kernel_source_hash() if sha is None else sha
    p = tmp_path / "hbm.md"
    p.write_text("# HBM bytes\n\nValues read by bench.py:\n\n"
                 f"- workload: `{workload}`\n- engine: `{engine}`\n- layout: `{layout}`\n"
                 f"- traffic_bytes_per_launch: `{value}`\n- kernel_source_sha256: `{sha}`\n")
    return str(p)


def test_traffic_read_when_everything_matches(tmp_path):
    p = summary(tmp_path)
    choice = [{"d": 2, "chi": 32, "engine": "valu", "layout": "compact"}]
    assert bench.measured_traffic("ea32", choice, path=p) == 2159731206.0
    assert bench.measured_traffic("ea32", path=p) == 2159731206.0


def test_traffic_null_on_any_mismatch(tmp_path):
    choice = [{"d": 2, "chi": 32, "engine": "valu", "layout": "compact"}]
    assert bench.measured_traffic("ea16", choice, path=summary(tmp_path)) is None
    assert bench.measured_traffic("ea32", choice, path=summary(tmp_path, sha="0" * 64)) is None
    assert bench.measured_traffic("ea32", choice, path=summary(tmp_path, engine="mfma")) is None
    assert bench.measured_traffic("ea32", choice, path=summary(tmp_path, layout="full")) is None
    assert bench.measured_traffic("ea32", [], path=summary(tmp_path)) is None
    assert bench.measured_traffic("ea32", choice * 2, path=summary(tmp_path)) is None
    assert bench.measured_traffic("ea32", choice, path=summary(tmp_path, value="n/a")) is None
    assert bench.measured_traffic("ea32", choice, path=str(tmp_path / "missing.md")) is None


def test_committed_summary_matches_the_current_sources():
    """The committed summary is for the sources as they are (else the bench
    line reports traffic null until the counters are taken again)."""
    choice = [{"d": 2, "chi": 32, "engine": "valu", "layout": "compact"}]
    assert bench.measured_traffic("ea32", choice) is not None
