"""Summaries of rocprofv3 output for the product kernel the bench line names.

    python -m paper_1905_01331_amd.rocprof_summary \\
        --bench BENCH.json --trace TRACE_DIR --fetch FETCH_DIR --write WRITE_DIR \\
        --copy-fetch CF_DIR --copy-write CW_DIR --command-file CMDS.txt \\
        --out-md profiles/NAME.md --out-json profiles/NAME.json

Inputs (CSV output of rocprofv3 with ``-o p --output-format csv``):
  * BENCH.json: the JSON line bench.py printed in the kernel-trace run; its
    ``roofline`` names the dominant kernel instantiation and how many times
    the profiled pass launched it.  The profiled pass is the last use of that
    kernel in the run, so its launches are the kernel's last dispatches;
  * TRACE_DIR: ``--kernel-trace --stats`` of the same bench command;
  * FETCH_DIR / WRITE_DIR: ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
    the same bench command (KiB per dispatch);
  * CF_DIR / CW_DIR: the same counters over ``bench.py --copy-calibration``,
    a plain elementwise copy (y = -x) of known size; the counter's reading for
    it against the bytes that copy must move gives the scale factor applied to
    the kernel's readings.

Writes a short Markdown summary (the commands, the kernel's durations from
the trace next to the bench's event timing, the top kernels of the stats,
the calibrated traffic per launch) and a JSON record of the traffic that
bench.py reads back while the product-kernel sources are unchanged
(``sources_sha256``).
"""
import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources a product kernel's memory traffic depends on
TRAFFIC_SOURCES = ["csrc/gemm_mfma.hip", "csrc/gemm_plain.hip", "csrc/gemm_tune.cpp", "csrc/common.h"]


def sources_sha256():
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _csv(d, suffix):
    path = os.path.join(d, "p_" + suffix + ".csv")
    if not os.path.exists(path):
        # rocprofv3 may place the files one directory further down
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith(suffix + ".csv"):
                    path = os.path.join(root, f)
    with open(path) as f:
        return list(csv.DictReader(f))


def trace_dispatches(d, kernel):
    rows = [r for r in _csv(d, "kernel_trace") if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]  # us


def counter_per_dispatch(d, kernel, counter):
    acc = {}
    for r in _csv(d, "counter_collection"):
        if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
            k = int(r["Dispatch_Id"])
            acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
    return [acc[k] for k in sorted(acc)]  # KiB


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--bench", required=True)
    p.add_argument("--trace", required=True)
    p.add_argument("--fetch")
    p.add_argument("--write")
    p.add_argument("--copy-fetch")
    p.add_argument("--copy-write")
    p.add_argument("--copy-json", help="the line bench.py --copy-calibration printed")
    p.add_argument("--command-file", required=True)
    p.add_argument("--out-md", required=True)
    p.add_argument("--out-json")
    p.add_argument("--top", type=int, default=12)
    a = p.parse_args()

    with open(a.bench) as f:
        bench = json.loads([l for l in f if l.startswith("{")][-1])
    rf = bench["roofline"]
    kernel, n = rf["kernel"], int(rf["launches"])
    durs = trace_dispatches(a.trace, kernel)
    last = durs[-n:]
    avg_pass = sum(last) / len(last)
    avg_all = sum(durs) / len(durs)
    stats = _csv(a.trace, "kernel_stats")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)

    L = []
    L.append(f"# Kernel {kernel}: {bench['config']['workload']} ({bench['dtype']})\n")
    L.append("Commands (from the repository root; rocprofv3 runs from /tmp with TMPDIR=/tmp):\n")
    with open(a.command_file) as f:
        L.append("```\n" + f.read().strip() + "\n```\n")
    L.append("## Duration of the dominant product kernel\n")
    L.append(f"* bench.py event timing (profiled pass, {n} launches): {rf['avg_launch_us']:.2f} us per launch")
    L.append(f"* kernel trace, same launches (the kernel's last {n} dispatches): {avg_pass:.2f} us per launch "
             f"({(avg_pass / rf['avg_launch_us'] - 1) * 100:+.1f} %)")
    L.append(f"* kernel trace, all {len(durs)} dispatches of the run (warm-up, launch-tuner candidates, timed "
             f"graph sweeps, profiled pass): {avg_all:.2f} us")
    L.append(f"* algorithmic work per launch: {rf['flops_per_launch'] / 1e9:.3f} GFLOP, "
             f"{rf['bytes_per_launch'] / 1e6:.2f} MB (operands read once, result written once); "
             f"intensity {rf['arith_intensity']} flop/B against a ridge of {rf['ridge']} flop/B")
    L.append(f"* roofline ({rf['bound']}): {rf['achieved']} {rf['unit']} of {rf['peak']} = {rf['frac']}\n")
    L.append(f"## Top kernels of the whole run (kernel-trace stats, {tot / 1e6:.1f} ms in all)\n")
    L.append("| kernel | calls | total ms | avg us | share |")
    L.append("|---|---:|---:|---:|---:|")
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:a.top]:
        name = r["Name"]
        short = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("ttn::", "")
        short = short.split("(")[0]
        L.append(f"| `{short[:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                 f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / tot * 100:.1f} % |")
    L.append("")

    rec = None
    if a.fetch and a.write and a.copy_fetch and a.copy_write and a.copy_json:
        with open(a.copy_json) as f:
            cj = json.loads([l for l in f if l.startswith("{")][-1])["copy_calibration"]
        ck = cj["kernel"]
        cf = counter_per_dispatch(a.copy_fetch, ck, "FETCH_SIZE")
        cw = counter_per_dispatch(a.copy_write, ck, "WRITE_SIZE")
        # the last copy launch: caches hold nothing of a 1 GiB source
        f_scale = cj["bytes_read"] / (cf[-1] * 1024.0)
        w_scale = cj["bytes_written"] / (cw[-1] * 1024.0)
        kf = counter_per_dispatch(a.fetch, kernel, "FETCH_SIZE")[-n:]
        kw = counter_per_dispatch(a.write, kernel, "WRITE_SIZE")[-n:]
        fetch = sum(kf) / len(kf) * 1024.0 * f_scale
        write = sum(kw) / len(kw) * 1024.0 * w_scale
        alg = rf["bytes_per_launch"]
        # keyed as bench.py looks it up: the workload's description and its precision
        rec = {"kernel": kernel, "workload": f"{bench['config']['workload']} {bench['config']['precision']}",
               "launches": n,
               "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
               "traffic_bytes_per_launch": fetch + write, "algorithmic_bytes_per_launch": alg,
               "fetch_scale": f_scale, "write_scale": w_scale, "sources_sha256": sources_sha256()}
        L.append("## HBM traffic of the dominant kernel (PMC)\n")
        L.append(f"* copy calibration: y = -x over {cj['bytes_read'] / 2**30:.2f} GiB; FETCH_SIZE reads "
                 f"{cf[-1] / 2**20:.3f} GiB (scale {f_scale:.4f}), WRITE_SIZE {cw[-1] / 2**20:.3f} GiB "
                 f"(scale {w_scale:.4f})")
        L.append(f"* per launch (mean over the profiled pass, scaled): fetch {fetch / 1e6:.2f} MB, "
                 f"write {write / 1e6:.2f} MB, total {(fetch + write) / 1e6:.2f} MB "
                 f"= {(fetch + write) / alg:.2f} x the algorithmic {alg / 1e6:.2f} MB")
        L.append(f"* sources hash {rec['sources_sha256'][:16]}\n")
    with open(a.out_md, "w") as f:
        f.write("\n".join(L))
    if rec and a.out_json:
        with open(a.out_json, "w") as f:
            json.dump(rec, f, indent=1)
    print("\n".join(L))


if __name__ == "__main__":
    main()
