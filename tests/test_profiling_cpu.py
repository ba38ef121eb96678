"""Host logic of the HBM traffic records (no GPU): counter CSVs to per-launch bytes with the
copy calibration, the choice of the iteration kernel of the stencil class, and the
kernel-source hash that decides whether a record still applies."""
import csv
import json
import os

from paper_1905_13408_amd import profiling


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, counter, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_summarize_scales_by_the_copy_and_picks_iteration_kernels(tmp_path):
    copy_bytes = 1 << 30
    # the copy reads 2^30 bytes but FETCH_SIZE shows half of that: fetch scale 2; writes exact
    _csv(tmp_path / "cf.csv", [("__amd_rocclr_copyBuffer(...)", "FETCH_SIZE", copy_bytes / 2 / 1024)])
    _csv(tmp_path / "cw.csv", [("__amd_rocclr_copyBuffer(...)", "WRITE_SIZE", copy_bytes / 1024)])
    fetch = [("void spg::k_fft_cols<512, 0>(...)", "FETCH_SIZE", 100.0),
             ("void spg::k_fft_cols<512, 0>(...)", "FETCH_SIZE", 300.0),
             ("void spg::k_prox_fft<512, 1, false, true, false>(...)", "FETCH_SIZE", 1000.0),
             ("void spg::k_prox_fft<512, 1, false, false, true>(...)", "FETCH_SIZE", 5.0),  # monitor: not counted
             ("void spg::k_prox_tv<1, true>(...)", "FETCH_SIZE", 7.0)]     # check launch: not counted
    write = [("void spg::k_fft_cols<512, 0>(...)", "WRITE_SIZE", 50.0),
             ("void spg::k_fft_cols<512, 0>(...)", "WRITE_SIZE", 50.0),
             ("void spg::k_prox_fft<512, 1, false, true, false>(...)", "WRITE_SIZE", 400.0),
             ("void spg::k_prox_fft<512, 1, false, false, true>(...)", "WRITE_SIZE", 3.0),
             ("void spg::k_prox_tv<1, true>(...)", "WRITE_SIZE", 9.0)]
    _csv(tmp_path / "f.csv", fetch)
    _csv(tmp_path / "w.csv", write)
    rec = profiling.summarize(tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "cf.csv", tmp_path / "cw.csv",
                              copy_bytes, "cmd")
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    y = rec["per_launch"]["fft_y_fwd"]
    assert y["launches"] == 2 and y["fetch_bytes"] == 2.0 * 200.0 * 1024 and y["write_bytes"] == 50.0 * 1024
    p = rec["per_launch"]["prox_tv"]
    assert p["launches"] == 1 and p["fetch_bytes"] == 2.0 * 1000.0 * 1024 and p["write_bytes"] == 400.0 * 1024
    assert rec["fused_x_transforms"] is True
    assert rec["kernel_source_sha256"] == profiling.source_sha256()


def test_record_applies_only_to_the_source_it_was_taken_on(tmp_path):
    rec = {"command": "c", "kernel_source_sha256": profiling.source_sha256(), "fused_x_transforms": True,
           "per_launch": {}}
    path = tmp_path / "rec.txt"
    path.write_text(json.dumps(rec))
    assert profiling.load(str(path)) is not None and profiling.record_fused(str(path))
    rec["kernel_source_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert profiling.load(str(path)) is None and not profiling.record_fused(str(path))
    assert profiling.load(str(tmp_path / "missing.txt")) is None


def test_source_hash_ignores_comments_and_blank_space(tmp_path):
    src = open(profiling.KERNEL_SOURCE).read()
    a = tmp_path / "a.hip"
    a.write_text("/* header */\n" + src.replace("\n", "\n\n") + "\n// end\n")
    assert profiling.source_sha256(str(a)) == profiling.source_sha256()
    b = tmp_path / "b.hip"
    b.write_text(src.replace("constexpr int PF_KB = 4;", "constexpr int PF_KB = 2;"))
    assert profiling.source_sha256(str(b)) != profiling.source_sha256()


def test_committed_record_is_well_formed():
    path = os.path.join(os.path.dirname(profiling.HERE), "profiles", "hbm_traffic_solve_512.txt")
    rec = json.loads(open(path).read())
    for cls in ["fft_y_fwd", "fft_z_weight", "fft_y_inv", "prox_tv"]:
        e = rec["per_launch"][cls]
        assert e["launches"] > 0 and e["fetch_bytes"] > 0 and e["write_bytes"] > 0
    assert len(rec["kernel_source_sha256"]) == 64 and rec["command"]
