"""Summary of a rocprofv3 kernel-trace statistics file (kernel_stats.csv from
`rocprofv3 --kernel-trace --stats --output-format csv`): the kernels by total
time, with their call counts, mean duration and share.

    python -m paper_2602_11092_amd.kernel_stats STATS_CSV OUT_TXT "<title>" "<command>" [ROWS]
"""
import csv
import sys

NOTE = ("(bench.py also runs the autotuner, whose parity gate and timing runs launch every candidate configuration a few\n"
        " times, and times each SLOS kernel on its own, so call counts exceed the timed replays)")
NOTE_CACHED = ("(bench.py takes the autotuner's choices from the cache file, written by an earlier bench.py run with the\n"
               " same option, and times each SLOS kernel on its own, so call counts exceed the timed replays)")


def summary(src, title, command, rows=16):
    recs = sorted(csv.DictReader(open(src)), key=lambda r: -float(r["TotalDurationNs"]))
    note = NOTE_CACHED if "--autotune-cache" in command else NOTE
    lines = ["rocprofv3 --kernel-trace --stats, %s" % title, "command: %s" % command, note, "",
             "%-100s %6s %10s %7s" % ("kernel", "calls", "avg_us", "pct")]
    for r in recs[:rows]:
        lines.append("%-100s %6s %10.2f %6.2f%%" % (r["Name"][:100], r["Calls"], float(r["AverageNs"]) / 1e3,
                                                    float(r["Percentage"])))
    return "\n".join(lines) + "\n"


def main(argv):
    src, out, title, command = argv[:4]
    text = summary(src, title, command, int(argv[4]) if len(argv) > 4 else 16)
    with open(out, "w") as f:
        f.write(text)
    print(text, end="")


if __name__ == "__main__":
    main(sys.argv[1:])
