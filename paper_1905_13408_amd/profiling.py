"""HBM traffic records from rocprofv3 counter runs.

``summarize`` turns two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
``bench.py`` (counter values in KiB per dispatch) plus the same two counters read on a
plain device copy of known size into per-kernel HBM bytes per launch.  The copy gives
the scale of each counter (bytes moved / counter bytes).  The record stores the
SHA-256 of the kernel source it was taken on (comments and blank space left out), so a
benchmark can tell whether the figures still describe the kernels it runs.

    python -m paper_1905_13408_amd.profiling FETCH.csv WRITE.csv COPY_FETCH.csv COPY_WRITE.csv \
        COPY_BYTES OUT.txt "command text"
"""
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "spg_kernels.hip")

# kernel-name prefixes (rocprofv3 names) -> kernel classes of the solver
CLASSES = [
    ("spg::k_fft_cols<512, 0>", "fft_y_fwd"), ("spg::k_fft_cols<512, 1>", "fft_y_inv"),
    ("spg::k_fft_zw<512, 2,", "fft_z_weight"), ("spg::k_dc_nyquist<512, false>", "dc_nyquist"),
    ("spg::k_c2r_x<256", "c2r_x"), ("spg::k_r2c_x<256", "r2c_x"), ("spg::k_prox_tv<", "prox_tv"),
]
# a trailing "true>" marks an objective/check instance of these kernels (not an iteration
# launch), except in the z pass, where it marks the streaming-load variant
KEEP_TRUE = ("spg::k_fft_zw<",)


FUSED = "spg::k_prox_fft<"  # stencil/prox kernel with the x-axis transforms inside


def source_sha256(path: str = KERNEL_SOURCE) -> str:
    """SHA-256 of the kernel source without its comments and blank space, so that a record
    stays valid across edits that cannot change the kernels."""
    import re

    with open(path) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)     # block comments
    txt = re.sub(r"//[^\n]*", " ", txt)                    # line comments
    txt = " ".join(txt.split())                            # whitespace runs
    return hashlib.sha256(txt.encode()).hexdigest()


def _per_kernel(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        agg[name].append(float(r["Counter_Value"]) * 1024.0)
    return agg


def _copy_scale(path, copy_bytes):
    agg = _per_kernel(path)
    vals = agg.get("__amd_rocclr_copyBuffer") or next(v for k, v in agg.items() if "copy" in k.lower())
    big = max(vals)
    return copy_bytes / big


def summarize(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, command):
    fs = _copy_scale(copy_fetch_csv, copy_bytes)
    wsc = _copy_scale(copy_write_csv, copy_bytes)
    fa, wa = _per_kernel(fetch_csv), _per_kernel(write_csv)
    out = {}
    for prefix, cls in CLASSES:
        keep = prefix.startswith(KEEP_TRUE)
        fv = [v for k, lst in fa.items() if k.startswith(prefix) and (keep or "true>" not in k[len(prefix):])
              for v in lst]
        wv = [v for k, lst in wa.items() if k.startswith(prefix) and (keep or "true>" not in k[len(prefix):])
              for v in lst]
        if cls == "prox_tv":
            # iteration launches only: the fused kernel where it ran, else the stencil kernel
            # outside its check mode (another instance)
            # (the objective-monitor instance, a trailing "true>", is not an iteration launch)
            fv = [v for k, lst in fa.items() if k.startswith(FUSED) and not k.endswith("true>") for v in lst]
            wv = [v for k, lst in wa.items() if k.startswith(FUSED) and not k.endswith("true>") for v in lst]
            if not fv:
                fv = [v for k, lst in fa.items() if k.startswith(prefix) and k.endswith("false>") for v in lst]
                wv = [v for k, lst in wa.items() if k.startswith(prefix) and k.endswith("false>") for v in lst]
        if fv and wv:
            # per launch, and in all (a pass over the map may be launched as several column
            # ranges)
            out[cls] = {"launches": len(fv), "fetch_bytes": fs * sum(fv) / len(fv),
                        "write_bytes": wsc * sum(wv) / len(wv),
                        "fetch_bytes_total": fs * sum(fv), "write_bytes_total": wsc * sum(wv)}
    fused = any(k.startswith(FUSED) for k in fa)
    return {"command": command, "kernel_source_sha256": source_sha256(), "fetch_scale": fs, "write_scale": wsc,
            "copy_bytes_each_way": copy_bytes, "fused_x_transforms": fused, "per_launch": out}


def load(path):
    """The record at `path`, or None if missing or taken on other kernel source."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.loads(f.read())
    if rec.get("kernel_source_sha256") != source_sha256():
        return None
    return rec


def record_fused(path) -> bool:
    """Whether the record at `path` was taken with the fused x-transform kernel."""
    rec = load(path)
    return bool(rec and rec.get("fused_x_transforms", False))


if __name__ == "__main__":
    a = sys.argv[1:]
    rec = summarize(a[0], a[1], a[2], a[3], float(a[4]), a[6])
    with open(a[5], "w") as f:
        f.write(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec, indent=1))
