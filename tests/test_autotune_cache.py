"""The autotuner's JSON cache (no GPU): defaults without an entry, stored
choices read back per device and workload, unknown keys ignored."""
from paper_2605_20497_amd import autotune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tuning.json")
    assert autotune.tuned_options("conv-6.9m", path=path, name="dev") == autotune.DEFAULT
    autotune.save({"dev": {"conv-6.9m": {"hash_log2": 11, "list_gate": 8, "ms": {"x": 1.0}},
                           autotune.stream_key(256, 262144): {"workers": 12}}}, path)
    got = autotune.tuned_options("conv-6.9m", path=path, name="dev")
    assert got == {"hash_log2": 11, "list_gate": 8, "workers": 8}
    assert autotune.tuned_options(autotune.stream_key(256, 262144), path=path, name="dev")["workers"] == 12
    assert autotune.tuned_options("conv-6.9m", path=path, name="other") == autotune.DEFAULT


def test_same_isa_under_another_name(tmp_path):
    """A process that sees the device under another marketing name (the
    runtime's name lookup can differ, e.g. under a profiler) still finds the
    entry stored for the same ISA, and never one of another ISA."""
    path = str(tmp_path / "tuning.json")
    autotune.save({"AMD Radeon Graphics (gfx950)": {"conv-6.9m": {"hash_log2": 11, "list_gate": 8}}}, path)
    got = autotune.tuned_options("conv-6.9m", path=path, name="AMD Instinct MI355X (gfx950)")
    assert (got["hash_log2"], got["list_gate"]) == (11, 8)
    assert autotune.tuned_options("conv-6.9m", path=path, name="AMD Instinct MI300X (gfx942)") == autotune.DEFAULT
    assert autotune.tuned_options("conv-6.9m", path=path, name="gfx950") == autotune.DEFAULT
