"""Render rocprofv3 SQLite output (``*_results.db``) as a short text summary:
per-kernel dispatch statistics, and per-kernel sums of hardware counters.

    python -m paper_2304_02731_amd.profsummary RESULTS.db [--lane-steps N]
"""
from __future__ import annotations

import argparse
import sqlite3


def short_name(name: str) -> str:
    """Kernel name without its argument list (and without the anonymous
    namespace's prefix, whose parenthesis would cut it short)."""
    return name.replace("(anonymous namespace)::", "").split("(")[0]


def kernel_stats(db: str):
    """(name, calls, total ns, average ns, percent) from the dispatch table."""
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), sum(end - start), avg(end - start) "
                     "from kernels group by name order by sum(end - start) desc").fetchall()
    tot = sum(r[2] for r in rows) or 1.0
    return [(n, k, t, a, 100.0 * t / tot) for n, k, t, a in rows]


def counters(db: str):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, counter_name, sum(value), count(distinct dispatch_id) "
                     "from counters_collection group by kernel_name, counter_name").fetchall()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--lane-steps", type=float, default=0.0,
                    help="divide FP64 counters of the propagation kernel by this")
    a = ap.parse_args()
    ks = kernel_stats(a.db)
    if ks:
        print("| kernel | calls | total ms | average ms | % |")
        print("|---|---|---|---|---|")
        for name, n, tot, avg, pct in ks:
            print("| %s | %d | %.3f | %.3f | %.2f |" % (short_name(name), n, tot / 1e6, avg / 1e6, pct))
    cs = counters(a.db)
    if cs:
        print()
        print("| kernel | counter | sum over dispatches | dispatches |")
        print("|---|---|---|---|")
        f64 = {}
        for kname, cname, v, nd in cs:
            short = short_name(kname)
            print("| %s | %s | %.6g | %d |" % (short, cname, v, nd))
            if "propagate" in short:
                f64[cname] = v
        if a.lane_steps and f64:
            g = lambda k: f64.get(k, 0.0)
            flop = 64.0 * (g("SQ_INSTS_VALU_ADD_F64") + g("SQ_INSTS_VALU_MUL_F64") +
                           g("SQ_INSTS_VALU_TRANS_F64") + 2.0 * g("SQ_INSTS_VALU_FMA_F64"))
            print()
            print("FP64 FLOP per lane-step (64 lanes x (ADD + MUL + TRANS + 2 FMA) / lane-steps): %.1f"
                  % (flop / a.lane_steps))
            for k in sorted(f64):
                print("  %s per lane-step: %.2f" % (k, 64.0 * f64[k] / a.lane_steps))


if __name__ == "__main__":
    main()
