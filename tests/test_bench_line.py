"""The benchmark's headline line (CPU): built from the figures of a real run
(profiles/bench_detail.json), it carries the required fields first and the
whole per-configuration summary within 4,000 characters, so that a log that
keeps only the tail of stdout still holds the complete line; with inflated
figures, summary parts are dropped rather than the required fields."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REQUIRED = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
            "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"]


def _line_from(detail):
    extras = {k: detail[k] for k in ("small", "precision", "widths", "hwc", "pyramid", "batch", "serving",
                                     "serving_small_frames") if k in detail}
    line = dict(detail["headline"])
    line["summary"] = bench.summarize(detail["forms"], extras, detail["fused_equals_2pass_bitwise"])
    return line


def _detail():
    with open(os.path.join(ROOT, "profiles", "bench_detail.json")) as f:
        return json.load(f)


def test_headline_of_a_real_run_fits_whole():
    line = _line_from(_detail())
    n_summary = len(line["summary"])
    text = bench.headline_text(line)
    assert len(text) <= bench.HEADLINE_MAX_CHARS
    parsed = json.loads(text)
    assert list(parsed)[:len(REQUIRED)] == REQUIRED
    assert len(parsed["summary"]) == n_summary, "a real run's summary should fit whole"
    for key in ("c2_us", "c1_us_per_call", "c3_batch64", "c4_us_per_image", "c5_mixed", "c5_640x480"):
        assert key in parsed["summary"], key
    r = parsed["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    c = parsed["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0


def test_oversized_summary_is_trimmed_not_the_headline():
    detail = _detail()
    line = _line_from(detail)
    # figures with many digits and a long workload name: the line grows past the limit
    line["config"]["workload"] = line["config"]["workload"] + " " + "x" * 600
    line["summary"]["c5_mixed"]["capacity_req_per_s"] = {f"policy_{i}": 123456.789012345 for i in range(40)}
    text = bench.headline_text(line)
    assert len(text) <= bench.HEADLINE_MAX_CHARS
    parsed = json.loads(text)
    assert list(parsed)[:len(REQUIRED)] == REQUIRED
    assert "c2_us" in parsed["summary"]
