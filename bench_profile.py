"""rocprofv3 measurements behind bench.py's roofline line.

    python3 bench_profile.py collect [--chunk C] [--out DIR]

runs, on a machine with the GPU, from the repository root:
  1. rocprofv3 --kernel-trace --stats on bench.py (per-kernel durations);
  2. rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, on bench.py;
  3. the same two counters on a plain 256 MiB device copy (torch copy_),
     whose true bytes are known, to scale the counters to bytes;
and writes DIR/traffic.json (HBM bytes per launch of each libqlc kernel,
tagged with the hash of the kernel sources) and
DIR/kernels_single_tensor_256MiB.md (the summary, with the commands, paths
relative to the repository root); both are then copied into profiles/,
where bench.py reads traffic.json while the kernel sources still match its
hash.  DIR defaults to profile_runs/ (raw rocprofv3 output, not committed).

    python3 bench_profile.py copy     # the calibration workload itself
    python3 bench_profile.py batched [--tuning C,LOG2_SEGMENT,LAG] [--out DIR]
        # kernel durations of the batched form on the 1152-shard workload
    python3 bench_profile.py sq [--kernel K] [--chunk C] [--out DIR]
        # SQ issue / stall counters of kernel K (default k_decode) on the
        # 256 MiB tensor (two --pmc passes of at most eight SQ counters each)
"""
from __future__ import annotations

import csv
import glob
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
OUT = "profile_runs"  # relative to ROOT; --out overrides
COPY_BYTES = 256 << 20


def copy_workload():
    import torch
    src = torch.randint(0, 255, (COPY_BYTES,), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copy done", flush=True)


def run(cmd, log):
    print("+", " ".join(cmd), flush=True)
    with open(log, "w") as f:
        r = subprocess.run(cmd, stdout=f, stderr=subprocess.STDOUT, cwd=ROOT, timeout=300)
    print("  rc=%d" % r.returncode, flush=True)
    if r.returncode != 0:
        with open(log) as f:
            print(f.read()[-3000:])
        raise SystemExit(r.returncode)


def counters(d):
    """Mean counter value per dispatch, by kernel short name."""
    per = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"]
            key = (name, r["Dispatch_Id"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        out.setdefault(name, []).append(v)
    return {k: sum(v) / len(v) for k, v in out.items()}


def short(name):
    return name.split("(")[0].replace("qlc::", "").replace("void ", "")


def kernel_stats(d):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    return rows


def collect(chunk):
    os.makedirs(OUT, exist_ok=True)
    bench = ["python3", "bench.py", "--steps", "5", "--warmup", "2", "--no-cpu-baseline",
             "--no-batched", "--no-serving", "--no-extra", "--chunk", str(chunk)]
    cmds = {}
    cmds["trace"] = ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv",
                     "-d", os.path.join(OUT, "trace"), "-o", "trace", "--"] + bench
    run(cmds["trace"], os.path.join(OUT, "trace.log"))
    vals = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        cmds[ctr] = ["rocprofv3", "--pmc", ctr, "--output-format", "csv",
                     "-d", os.path.join(OUT, ctr), "-o", ctr, "--"] + bench
        run(cmds[ctr], os.path.join(OUT, ctr + ".log"))
        vals[ctr] = counters(os.path.join(OUT, ctr))
        cmds[ctr + "_copy"] = ["rocprofv3", "--pmc", ctr, "--output-format", "csv",
                               "-d", os.path.join(OUT, ctr + "_copy"), "-o", ctr, "--",
                               "python3", "bench_profile.py", "copy"]
        run(cmds[ctr + "_copy"], os.path.join(OUT, ctr + "_copy.log"))
        vals[ctr + "_copy"] = counters(os.path.join(OUT, ctr + "_copy"))

    def copy_reading(ctr):
        cands = [v for k, v in vals[ctr + "_copy"].items() if "copy" in k.lower()]
        return max(cands) if cands else None

    f_read = copy_reading("FETCH_SIZE")
    f_write = copy_reading("WRITE_SIZE")
    scale_r = COPY_BYTES / (f_read * 1024.0) if f_read else None
    scale_w = COPY_BYTES / (f_write * 1024.0) if f_write else None

    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash
    kernels = {}
    for name, fetch_kb in vals["FETCH_SIZE"].items():
        s = short(name)
        if not s.startswith("k_"):
            continue
        write_kb = vals["WRITE_SIZE"].get(name, 0.0)
        rd = fetch_kb * 1024.0 * scale_r if scale_r else None
        wr = write_kb * 1024.0 * scale_w if scale_w else None
        kernels[s] = {"fetch_kb": fetch_kb, "write_kb": write_kb, "read_bytes": rd,
                      "write_bytes": wr,
                      "bytes_per_launch": (rd + wr) if rd is not None and wr is not None else None}
    stats = kernel_stats(os.path.join(OUT, "trace"))
    for r in stats:
        nm = short(r.get("Name", ""))
        if nm in kernels:
            kernels[nm]["avg_us"] = float(r["AverageNs"]) / 1e3
            kernels[nm]["calls"] = int(r["Calls"])
    rec = {"source_hash": kernel_source_hash(), "chunk_symbols": chunk,
           "copy_bytes": COPY_BYTES, "copy_fetch_kb": f_read, "copy_write_kb": f_write,
           "read_scale": scale_r, "write_scale": scale_w, "kernels": kernels,
           "commands": {k: " ".join(v) for k, v in cmds.items()},
           "date": time.strftime("%Y-%m-%d %H:%M:%S")}
    with open(os.path.join(OUT, "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)

    lines = ["# libqlc kernels on the single 256 MiB tensor (8192x32768 Laplace e4m3)", "",
             "Kernel durations: `%s` (run from the repository root)" % " ".join(cmds["trace"]),
             "", "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in stats:
        nm = short(r.get("Name", ""))
        if not nm.startswith("k_"):
            continue
        avg = float(r["AverageNs"]) / 1e3
        lines.append("| %s | %s | %.2f | %.2f | %.2f |" % (
            nm, r["Calls"], avg, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
    lines += ["", "HBM traffic per launch: `%s` and `%s`, scaled by a plain %d-byte copy "
              "(`%s`, `%s`): read scale %.4f, write scale %.4f" % (
                  " ".join(cmds["FETCH_SIZE"]), " ".join(cmds["WRITE_SIZE"]), COPY_BYTES,
                  " ".join(cmds["FETCH_SIZE_copy"]), " ".join(cmds["WRITE_SIZE_copy"]),
                  scale_r or 0, scale_w or 0),
              "", "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | write MB |",
              "|---|---|---|---|---|"]
    for k, v in sorted(kernels.items()):
        lines.append("| %s | %.0f | %.0f | %.1f | %.1f |" % (
            k, v["fetch_kb"], v["write_kb"], (v["read_bytes"] or 0) / 1e6,
            (v["write_bytes"] or 0) / 1e6))
    lines += ["", "Kernel source hash: %s" % rec["source_hash"]]
    with open(os.path.join(OUT, "kernels_single_tensor_256MiB.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def collect_batched(tuning):
    """Kernel durations of the batched form on the 1152-shard workload, at a
    fixed tuning (no autotuner calls in the trace)."""
    os.makedirs(OUT, exist_ok=True)
    cmd = ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv",
           "-d", os.path.join(OUT, "trace_batched"), "-o", "trace", "--",
           "python3", "bench.py", "--steps", "3", "--warmup", "1", "--no-cpu-baseline",
           "--no-serving", "--no-extra", "--batched-tuning", tuning]
    run(cmd, os.path.join(OUT, "trace_batched.log"))
    stats = kernel_stats(os.path.join(OUT, "trace_batched"))
    c, l2, lag = tuning.split(",")
    lines = ["# libqlc batched kernels on 1152 shards (1-32 MiB, 10.25 GiB)", "",
             "Chunk %s symbols, segments of 2^%s symbols, lag %s.  Kernel durations: `%s` "
             "(run from the repository root).  Each call of k_encode_batched / "
             "k_decode_batched processes all 1152 shards; the single-tensor kernels "
             "of the same run (the 256 MiB tensor and the plain per-shard comparison) "
             "are listed for reference." % (c, l2, lag, " ".join(cmd)), "",
             "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: short(r.get("Name", ""))):
        nm = short(r.get("Name", ""))
        if not nm.startswith("k_"):
            continue
        lines.append("| %s | %s | %.2f | %.2f | %.2f |" % (
            nm, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3))
    with open(os.path.join(OUT, "kernels_batched_1152_shards.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_PASSES = (
    ["SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
     "SQ_INSTS_LDS", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_ANY"],
    ["SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT",
     "SQ_LDS_IDX_ACTIVE", "SQ_LDS_ADDR_CONFLICT", "SQ_INSTS_VMEM_RD", "SQ_ACTIVE_INST_VMEM"],
)


def collect_sq(chunk, kernel="k_decode"):
    """Per-launch SQ counters of one kernel, summed over the device, and
    per-wave figures derived from them (wave-cycle counters are in units of
    four cycles)."""
    os.makedirs(OUT, exist_ok=True)
    bench = ["python3", "bench.py", "--steps", "3", "--warmup", "1", "--no-cpu-baseline",
             "--no-batched", "--no-serving", "--no-extra", "--chunk", str(chunk)]
    vals, cmds = {}, []
    for i, ctrs in enumerate(SQ_PASSES):
        d = os.path.join(OUT, "sq%d" % (i + 1))
        cmd = ["rocprofv3", "--pmc"] + ctrs + ["--output-format", "csv", "-d", d,
                                               "-o", "sq%d" % (i + 1), "--"] + bench
        cmds.append(cmd)
        run(cmd, d + ".log")
        per = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if short(r["Kernel_Name"]).split("<")[0] != kernel:
                    continue
                key = (r["Counter_Name"], r["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        for (c, _), v in per.items():
            vals.setdefault(c, []).append(v)
    v = {c: sum(x) / len(x) for c, x in vals.items()}
    waves = v.get("SQ_WAVES", 0.0) or 1.0
    life = v.get("SQ_WAVE_CYCLES", 0.0) / waves or 1.0
    lines = ["# SQ counters of %s on the single 256 MiB tensor (C = %d)" % (kernel, chunk), "",
             "Commands (run from the repository root): " +
             "; ".join("`%s`" % " ".join(c) for c in cmds), "",
             "| counter | per launch (device total) | per wave | % of wave lifetime |",
             "|---|---|---|---|"]
    for c in SQ_PASSES[0] + SQ_PASSES[1]:
        if c not in v:
            continue
        pw = v[c] / waves
        frac = ("%.1f" % (100.0 * pw / life)) if c.startswith(("SQ_ACTIVE", "SQ_WAIT")) else ""
        lines.append("| %s | %.4g | %.4g | %s |" % (c, v[c], pw, frac))
    if v.get("SQ_LDS_IDX_ACTIVE"):
        lines += ["", "LDS bank-conflict stall cycles / LDS indexed-active cycles: %.3f" % (
            v.get("SQ_LDS_BANK_CONFLICT", 0.0) / v["SQ_LDS_IDX_ACTIVE"])]
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash
    lines += ["", "Kernel source hash: %s" % kernel_source_hash()]
    with open(os.path.join(OUT, "%s_sq_counters_256MiB.md" % kernel), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "copy":
        copy_workload()
    elif len(sys.argv) > 1 and sys.argv[1] == "sq":
        if "--out" in sys.argv:
            OUT = sys.argv[sys.argv.index("--out") + 1]
        chunk = int(sys.argv[sys.argv.index("--chunk") + 1]) if "--chunk" in sys.argv else 2048
        os.environ["TMPDIR"] = "/tmp"
        os.chdir(ROOT)
        kernel = sys.argv[sys.argv.index("--kernel") + 1] if "--kernel" in sys.argv else "k_decode"
        collect_sq(chunk, kernel)
    elif len(sys.argv) > 1 and sys.argv[1] == "batched":
        if "--out" in sys.argv:
            OUT = sys.argv[sys.argv.index("--out") + 1]
        os.environ["TMPDIR"] = "/tmp"
        os.chdir(ROOT)
        collect_batched(sys.argv[sys.argv.index("--tuning") + 1] if "--tuning" in sys.argv
                        else "2048,19,0")
    else:
        chunk = 2048
        if "--chunk" in sys.argv:
            chunk = int(sys.argv[sys.argv.index("--chunk") + 1])
        if "--out" in sys.argv:
            OUT = sys.argv[sys.argv.index("--out") + 1]
        os.chdir("/tmp")
        os.environ["TMPDIR"] = "/tmp"
        os.chdir(ROOT)
        collect(chunk)
