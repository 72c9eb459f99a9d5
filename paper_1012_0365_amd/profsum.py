"""Short markdown summaries of rocprofv3 output, as kept in profiles/.

    python -m paper_1012_0365_amd.profsum stats <kernel_stats.csv> "<command>"
        top kernels by total time (from --kernel-trace --stats)
    python -m paper_1012_0365_amd.profsum traffic <dir> <family> <kernel-substring> <source> [more kernel substrings]
        HBM bytes per dispatch from the PMC runs in <dir>: pmc_FETCH_SIZE/,
        pmc_WRITE_SIZE/ (the workload) and pmcc_FETCH_SIZE/, pmcc_WRITE_SIZE/
        (bench.py --workload copy, a 256 MiB device copy that calibrates each
        counter); ends with the machine-readable line bench.py reads, tied to
        the SHA-256 of the kernel's source file.
"""

import csv
import hashlib
import os
import re
import sys

COPY_KIB = 256 * 1024


def short(name: str) -> str:
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"\(int, .*\)$", "(...)", name)
    return name.replace("blws::", "")


def stats(path, cmd):
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"Command: `{cmd}`\n")
    print(f"Total kernel time: {total / 1e6:.2f} ms over {sum(int(r['Calls']) for r in rows)} "
          "dispatches\n")
    print("| kernel | calls | total ms | avg us | min us | max us | % |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        print(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
              f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")


def counter(d, key):
    rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
    return [float(r["Counter_Value"]) for r in rows if key in r["Kernel_Name"]]


def traffic(d, family, key, source, *more):
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        scale[c] = COPY_KIB / counter(os.path.join(d, "pmcc_" + c), "copyBuffer")[0]
    print("| counter | reads for the 256 MiB copy (KiB) | scale factor |")
    print("|---|---:|---:|")
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        print(f"| {c} | {COPY_KIB / scale[c]:.2f} | {scale[c]:.5f} |")
    print()
    print("| kernel | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | scaled traffic (MB) |")
    print("|---|---:|---:|---:|---:|")
    t = None
    for kk in (key,) + more:
        f = counter(os.path.join(d, "pmc_FETCH_SIZE"), kk)
        w = counter(os.path.join(d, "pmc_WRITE_SIZE"), kk)
        fa, wa = sum(f) / len(f), sum(w) / len(w)
        tk = (fa * scale["FETCH_SIZE"] + wa * scale["WRITE_SIZE"]) * 1024
        if t is None:
            t = tk
        print(f"| `{kk}` | {len(f)} | {fa:.2f} | {wa:.2f} | {tk / 1e6:.3f} |")
    print()
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sha = hashlib.sha256(open(os.path.join(here, source), "rb").read()).hexdigest()
    print(f"traffic: kernel={family} bytes_per_launch={int(round(t))} source={source} sha256={sha}")


def main():
    if len(sys.argv) >= 4 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 6 and sys.argv[1] == "traffic":
        traffic(*sys.argv[2:])
    else:
        print(__doc__, file=sys.stderr)
        sys.exit(2)


if __name__ == "__main__":
    main()
