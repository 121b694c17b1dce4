"""Summaries of rocprofv3 result databases (kernel times, counters, traffic).

    python -m paper_1904_02603_amd.rocprof_summary times  RESULTS.db [N]
    python -m paper_1904_02603_amd.rocprof_summary counters RESULTS.db
    python -m paper_1904_02603_amd.rocprof_summary traffic FETCH.db WRITE.db KERNEL_SUBSTRING

`traffic` scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the kernel by
what the same counters read for the plain 512 MiB device-to-device copy that
``bench.py --calibrate-copy`` runs first (512 MiB read and 512 MiB written).
"""
import collections
import sqlite3
import sys

COPY_BYTES = 512 * 1024 * 1024


def times(db, n=25):
    c = sqlite3.connect(db)
    q = ("select name, count(*), sum(end-start)/1e3, avg(end-start)/1e3, max(vgpr_count), "
         "max(accum_vgpr_count), max(lds_size), max(scratch_size) from kernels group by name "
         "order by sum(end-start) desc limit %d" % n)
    print("%-72s %5s %10s %9s %5s %5s %6s %4s" % ("kernel", "calls", "total_us", "avg_us", "vgpr", "agpr",
                                                 "lds", "scr"))
    for r in c.execute(q):
        print("%-72s %5d %10.1f %9.2f %5d %5d %6d %4d" % ((r[0][:72],) + tuple(r[1:])))


def _per_dispatch(db, counter):
    c = sqlite3.connect(db)
    q = ("select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name=? "
         "group by kernel_name, dispatch_id order by dispatch_id")
    d = collections.defaultdict(list)
    for name, _, v in c.execute(q, (counter,)):
        d[name].append(v)
    return d


def _first_copy(db, counter):
    # the calibration copy (device to device, 512 MiB) is the first blit-copy
    # dispatch of the run
    c = sqlite3.connect(db)
    q = ("select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name=? "
         "and kernel_name like '%copyBuffer%' group by kernel_name, dispatch_id order by dispatch_id limit 1")
    r = list(c.execute(q, (counter,)))
    return (r[0][0], r[0][2]) if r else (None, None)


def counters(db):
    c = sqlite3.connect(db)
    names = [r[0] for r in c.execute("select distinct counter_name from counters_collection")]
    for cn in names:
        d = _per_dispatch(db, cn)
        for k, v in sorted(d.items(), key=lambda x: -sum(x[1]))[:12]:
            print("%-14s %-64s n=%-3d avg/dispatch=%.4g" % (cn, k[:64], len(v), sum(v) / len(v)))


def traffic(fetch_db, write_db, kernel, first=None):
    f = _per_dispatch(fetch_db, "FETCH_SIZE")
    w = _per_dispatch(write_db, "WRITE_SIZE")
    if first is not None:  # only the first `first` dispatches of each kernel
        f = {k: v[:first] for k, v in f.items()}
        w = {k: v[:first] for k, v in w.items()}
    ck, cf = _first_copy(fetch_db, "FETCH_SIZE")
    _, cw = _first_copy(write_db, "WRITE_SIZE")
    if ck is None:
        raise SystemExit("no calibration copy found (run bench.py with --calibrate-copy)")
    sf, sw = COPY_BYTES / (cf * 1024.0), COPY_BYTES / (cw * 1024.0)
    print("calibration: %s, 512 MiB copy reads FETCH_SIZE %.6g KiB (scale %.4f), WRITE_SIZE %.6g KiB "
          "(scale %.4f)" % (ck, cf, sf, cw, sw))
    for k in f:
        if kernel in k:
            fr = sum(f[k]) / len(f[k])
            wr = sum(w.get(k, [0.0])) / max(1, len(w.get(k, [1])))
            print("%s\n  per dispatch: FETCH_SIZE %.6g KiB, WRITE_SIZE %.6g KiB -> read %.4g B, written %.4g B, "
                  "total %.4g B (%d dispatches)" % (k, fr, wr, fr * 1024 * sf, wr * 1024 * sw,
                                                    fr * 1024 * sf + wr * 1024 * sw, len(f[k])))


if __name__ == "__main__":
    if sys.argv[1] == "times":
        times(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25)
    elif sys.argv[1] == "counters":
        counters(sys.argv[2])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]) if len(sys.argv) > 5 else None)
