"""Turn a rocprofv3 --kernel-trace --stats kernel_stats.csv into the short
markdown table kept in profiles/ (top kernels by total time).

    python profiles/summarize.py <kernel_stats.csv> "<command that produced it>" > out.md
"""

import csv
import re
import sys


def short(name: str) -> str:
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"\(int, .*\)$", "(...)", name)
    return name.replace("blws::", "")


def main():
    path, cmd = sys.argv[1], sys.argv[2]
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


if __name__ == "__main__":
    main()
