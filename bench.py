"""Throughput of the fused RLBD stream-and-collide step on one MI355X.

Headline workload: a 256^3 periodic box in mixed precision (float32
populations; moments, Landau frame and equilibrium coefficients in
float64), smooth random fields with |v| <= 0.6 and eta/s = 0.5.  The same
box is also timed in full float64, and both precisions are timed again
with the second-order model of Appendix A (66 points instead of 128).  A
step is one launch of the fused gather-moments-Landau-equilibrium-collision
kernel over every cell; inputs are resident in HBM before timing starts.

Prints one JSON line (rank 0).  --gpus > 1 is not supported: the program
runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

# The serving leg's server runs four streams that should each have a
# hardware queue of their own; HIP gives a process four by default, and
# streams made earlier in the process (torch's, the box legs') would then
# share queues with them (measured: serving p50 0.51 s instead of 0.30 s).
# Read by the HIP runtime when it starts, so set before torch is imported
# (raised to 8 unless the environment already asks for more).
try:
    _queues = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
except ValueError:
    _queues = 0
os.environ["GPU_MAX_HW_QUEUES"] = str(max(_queues, 8))

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

HBM_PEAK_GBS = 8000.0
# why the random-field box runs at |v| <= 0.6 (tests/test_oracle_stability.py)
VMAX_NOTE = ("; |v|<=0.6 instead of 0.8 because at 0.8 the scheme itself turns non-physical (n<0, |v|>=1) "
             "within two steps on the oracle (64^3, seed 3, eta/s=0.5), its expanded equilibrium being "
             "strongly negative at such speeds")
Q_OF_ORDER = {3: 128, 2: 66}


ACCESS = {"pull": 0, "aa_even": 1, "aa_odd": 2}   # the kernels' access template argument


def kernel_name(order, precision, edge, access="pull"):
    """The step kernel the library launches for a box of this edge (two-buffer
    pull, or the even or odd step of the in-place AA pattern)."""
    a = ACCESS[access]
    two_lane = precision == "fp64" or edge % 64 != 0
    if access == "aa_odd" and two_lane and edge > 6:
        a = 3   # the odd step's form for boxes wider than the largest shift
    if access == "aa_odd" and not two_lane and 256 % edge == 0:
        a = 4   # the odd step with stores rotated through LDS (rows wholly in a block)
    if precision == "fp64":
        return "k_step<Model<%d>, double, false, %d>" % (order, a)
    return ("k_step_row<Model<%d>, float, false, %d>" if edge % 64 == 0
            else "k_step<Model<%d>, float, false, %d>") % (order, a)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--edge", type=int, default=256)
    ap.add_argument("--vmax", type=float, default=0.6)
    ap.add_argument("--eta-s", type=float, default=0.5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tubes", action="store_true")
    ap.add_argument("--no-second-order", action="store_true")
    ap.add_argument("--no-walls", action="store_true")
    ap.add_argument("--no-aa", action="store_true")
    ap.add_argument("--no-largest", action="store_true", help="skip the largest-box AA leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the full-length runs of the 128^3 float64 and 256^3 mixed configurations")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/*.txt from the rocprofv3 CSV output under DIR (no GPU needed)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 4 GiB device copy (for calibrating traffic counters)")
    return ap.parse_args()


def copy_bandwidth():
    """GB/s (read + write) of a plain 4 GiB device copy, timed with HIP
    events: the practical streaming ceiling next to the 8 TB/s peak."""
    import torch
    n = 4 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n / (ms * 1e-3) / 1e9


def stream_ceiling():
    """What this device streams in practice: the best of a few launch shapes
    of the hand-written copy, read-only and write-only kernels in
    libstream_probe.so over 4 GiB buffers (GB/s: bytes read plus written per
    second; the copy counts both)."""
    import ctypes
    import torch
    from paper_1301_3423_amd import build as _b
    if not os.path.exists(_b.PROBE_OUT):
        raise RuntimeError("libstream_probe.so is not built (python -m paper_1301_3423_amd.build)")
    lib = ctypes.CDLL(_b.PROBE_OUT)
    f = lib.stream_probe_ms
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    n = 4 << 30
    grids = (2048, 8192)
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(max(grids) * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    out = {}
    for kind, name, factor in ((0, "copy", 2), (1, "copy_nontemporal", 2), (2, "read", 1), (3, "write", 1)):
        best = None
        for unroll in (1, 2, 4, 8):
            for grid in grids:
                ms = f(kind, unroll, grid, src.data_ptr(), dst.data_ptr(), sink.data_ptr(), n, 4, st.cuda_stream)
                if ms <= 0:
                    raise RuntimeError("stream probe failed (kind %d, unroll %d, grid %d): %g" % (kind, unroll, grid, ms))
                gbs = factor * n / (ms * 1e-3) / 1e9
                if best is None or gbs > best[0]:
                    best = (gbs, unroll, grid)
        out[name + "_GBps"] = round(best[0], 1)
        out[name + "_shape"] = "%d x 16 B in flight per thread, %d workgroups of 256" % (best[1], best[2])
    del src, dst, sink
    torch.cuda.empty_cache()
    out["note"] = ("hand-written streaming kernels over 4 GiB (csrc/stream_probe.hip), the best launch shape of "
                   "1-8 16-byte vectors in flight per thread and 2048 or 8192 workgroups, shortest of 4 launches")
    return out


def copy_calibration():
    """A plain device-to-device copy of known size: 4 GiB read + 4 GiB
    written per launch, three launches."""
    import torch
    n = 4 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)


# ---- rocprofv3 summaries (profiles/*.txt) ---------------------------------
#
# The commands below are run from /tmp with TMPDIR=/tmp on the GPU ($R is the
# repository root, $OUT an output directory); `python bench.py
# --summarize-profiles $OUT` then reads their CSV output and writes one
# summary per kernel.
_BOX_FLAGS = "--no-cpu --no-tubes --no-largest --no-configs --serve-requests 0"
_TUBE_FLAGS = "--no-fp64 --no-second-order --no-walls --no-aa --no-configs --serve-requests 0 --no-cpu"
PROFILE_RUNS = {
    "trace": "rocprofv3 --kernel-trace --stats -f csv -d $OUT/trace -o run -- "
             "python3 $R/bench.py --steps 20 --warmup 2 " + _BOX_FLAGS,
    "pmc_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d $OUT/pmc_fetch -o run -- "
                 "python3 $R/bench.py --steps 3 --warmup 1 " + _BOX_FLAGS,
    "pmc_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d $OUT/pmc_write -o run -- "
                 "python3 $R/bench.py --steps 3 --warmup 1 " + _BOX_FLAGS,
    "trace_tubes": "rocprofv3 --kernel-trace --stats -f csv -d $OUT/trace_tubes -o run -- "
                   "python3 $R/bench.py --steps 2 --warmup 1 " + _TUBE_FLAGS,
    "pmc_tubes_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d $OUT/pmc_tubes_fetch -o run -- "
                       "python3 $R/bench.py --steps 2 --warmup 1 " + _TUBE_FLAGS,
    "pmc_tubes_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d $OUT/pmc_tubes_write -o run -- "
                       "python3 $R/bench.py --steps 2 --warmup 1 " + _TUBE_FLAGS,
    "pmc_copy_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d $OUT/pmc_copy_fetch -o run -- "
                      "python3 $R/bench.py --copy-calibration",
    "pmc_copy_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d $OUT/pmc_copy_write -o run -- "
                      "python3 $R/bench.py --copy-calibration",
}
_BOX_WORKLOAD = "256^3 periodic box, random fields |v|<=0.6 (seed 3), T=1+-10%, eta/s=0.5 (bench.py defaults)"


def _profiled_kernels():
    """(file stem, kernel, description, algorithmic bytes per launch, extra
    workload note) of every step kernel the box legs launch at 256^3."""
    cells = 256 ** 3
    fluid = 256 * (256 - 12) * 256
    out = []
    for order, tag in ((3, ""), (2, "_order2")):
        for prec, stem in (("mixed", "k_step_row_f32_256cube"), ("fp64", "k_step_f64_256cube")):
            b = 4 if prec == "mixed" else 8
            what = ("%s-order %s step kernel" % ("third" if order == 3 else "second",
                    "mixed-precision (float32 populations, float64 moments/frame)" if prec == "mixed" else "float64"))
            out.append((stem + tag, kernel_name(order, prec, 256), what, 2 * Q_OF_ORDER[order] * b * cells, None))
            if order == 3:
                for acc in ("aa_even", "aa_odd"):
                    out.append((stem + "_" + acc, kernel_name(3, prec, 256, acc),
                                what + ", %s step of the in-place AA pattern" % acc.split("_")[1],
                                2 * 128 * b * cells, None))
    out.append(("k_step_row_f32_256cube_walls", "k_step_row<Model<3>, float, true, 0>",
                "third-order mixed step kernel with solid walls", 2 * 128 * 4 * fluid,
                "solid slabs of 6 cells at both y ends (4.7% solid); algorithmic bytes counted over the fluid "
                "cells (solid lanes leave at once)"))
    return out


def _short_kernel(name):
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    n = n.replace("rlb::", "")
    depth = 0
    for k, ch in enumerate(n):   # cut the argument list: the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:k]
    return n


def _read_csv(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _find(run_dir, suffix):
    for root, _, files in os.walk(run_dir):
        for f in sorted(files):
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError("no *%s under %s" % (suffix, run_dir))


def _dispatch_counters(run_dir, counter):
    """{kernel: [value per dispatch]} of one counter (KiB), in dispatch order."""
    rows = _read_csv(_find(run_dir, "counter_collection.csv"))
    per = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        per.setdefault(_short_kernel(r["Kernel_Name"]), []).append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return {k: [v for _, v in sorted(vs)] for k, vs in per.items()}


def _dispatch_times(run_dir):
    """{kernel: [duration ms per dispatch]} from a kernel trace."""
    rows = _read_csv(_find(run_dir, "kernel_trace.csv"))
    per = {}
    for r in rows:
        per.setdefault(_short_kernel(r["Kernel_Name"]), []).append(
            (int(r["Dispatch_Id"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6))
    return {k: [v for _, v in sorted(vs)] for k, vs in per.items()}


def summarize_profiles(prof_root):
    """Writes profiles/<kernel>.txt from the CSV output of PROFILE_RUNS."""
    from paper_1301_3423_amd.build import source_digest
    digest = source_digest()
    copy_fetch = _dispatch_counters(os.path.join(prof_root, "pmc_copy_fetch"), "FETCH_SIZE")
    copy_write = _dispatch_counters(os.path.join(prof_root, "pmc_copy_write"), "WRITE_SIZE")
    ck = [k for k in copy_fetch if "copyBuffer" in k]
    if not ck:
        raise RuntimeError("no device copy kernel in the calibration runs: %s" % sorted(copy_fetch))
    ck = ck[0]
    nbytes = 4 << 30
    cf = float(np.median(copy_fetch[ck]))
    cw = float(np.median(copy_write[ck]))
    f_fetch = nbytes / (cf * 1024.0)
    f_write = nbytes / (cw * 1024.0)
    cmds = lambda keys: "".join("#   %s\n" % PROFILE_RUNS[k] for k in keys)
    calib = ("# calibration: a plain 4 GiB device copy (%s) reads FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB per "
             "launch,\n#   so bytes = FETCH_SIZE KiB * 1024 * %.4f and bytes = WRITE_SIZE KiB * 1024 * %.4f\n"
             % (ck, cf, cw, f_fetch, f_write))
    head = "# commands (run from /tmp with TMPDIR=/tmp; R is the repository root, OUT an output directory):\n"
    tail = "#   then, on any host: python bench.py --summarize-profiles $OUT\n"
    written = []
    times = _dispatch_times(os.path.join(prof_root, "trace"))
    fetch = _dispatch_counters(os.path.join(prof_root, "pmc_fetch"), "FETCH_SIZE")
    write = _dispatch_counters(os.path.join(prof_root, "pmc_write"), "WRITE_SIZE")
    for stem, kern, what, alg, note in _profiled_kernels():
        if kern not in times or kern not in fetch or kern not in write:
            continue
        t = times[kern]
        avg = float(np.mean(t))
        fk, wk = float(np.mean(fetch[kern])), float(np.mean(write[kern]))
        rb, wb = fk * 1024 * f_fetch, wk * 1024 * f_write
        text = ("# rocprofv3 summary: %s %s\n# workload: %s%s\n" % (what, kern, _BOX_WORKLOAD,
                                                                     "; " + note if note else "")
                + head + cmds(["trace", "pmc_fetch", "pmc_write", "pmc_copy_fetch", "pmc_copy_write"]) + tail + calib
                + "# trace: %d dispatches avg %.4f ms (min %.4f, max %.4f)\n" % (len(t), avg, min(t), max(t))
                + "kernel: %s\nedge: 256\ncells: %d\ndispatches_traced: %d\nkernel_avg_ms: %.4f\n"
                  % (kern, 256 ** 3, len(t), avg)
                + "fetch_size_kib_per_dispatch: %.1f\nwrite_size_kib_per_dispatch: %.1f\n" % (fk, wk)
                + "read_bytes_per_launch: %d\nwrite_bytes_per_launch: %d\ntraffic_bytes_per_launch: %d\n"
                  % (rb, wb, rb + wb)
                + "algorithmic_bytes_per_launch: %d\n" % alg
                + "traffic_over_algorithmic: %.4f\nread_over_algorithmic: %.4f\nwrite_over_algorithmic: %.4f\n"
                  % ((rb + wb) / alg, 2 * rb / alg, 2 * wb / alg)
                + "achieved_algorithmic_GBps_at_avg: %.1f\nmeasured_traffic_GBps_at_avg: %.1f\n"
                  % (alg / (avg * 1e-3) / 1e9, (rb + wb) / (avg * 1e-3) / 1e9)
                + "source_sha256: %s\n" % digest)
        path = os.path.join(REPO, "profiles", stem + ".txt")
        with open(path, "w") as fh:
            fh.write(text)
        written.append(path)
    times = _dispatch_times(os.path.join(prof_root, "trace_tubes"))
    fetch = _dispatch_counters(os.path.join(prof_root, "pmc_tubes_fetch"), "FETCH_SIZE")
    write = _dispatch_counters(os.path.join(prof_root, "pmc_tubes_write"), "WRITE_SIZE")
    from paper_1301_3423_amd import inputs
    cells = sum(t["N"] for t in inputs.tube_batch(512, 4))
    for prec, stem, kern in (("mixed", "k_tubes_f32_512tubes", "k_tubes<Model<3>, float>"),
                             ("fp64", "k_tubes_f64_512tubes", "k_tubes<Model<3>, double>")):
        if kern not in times or kern not in fetch or kern not in write:
            continue
        # the bench launches 2 warm-up steps, then the 500 timed ones: the longest dispatch
        k = int(np.argmax(times[kern]))
        ms = times[kern][k]
        b = 4 if prec == "mixed" else 8
        alg = cells * 500 * 2 * 128 * b
        rb, wb = fetch[kern][k] * 1024 * f_fetch, write[kern][k] * 1024 * f_write
        text = ("# rocprofv3 summary: third-order tube batch kernel %s\n" % kern
                + "# workload: 512 shock tubes 1x1xN, N~U{200..4000} (%d cells), T_L/T_R~U(1.1,2), eta/s in "
                  "{0.01,0.05,0.1,0.2,0.5}, seed 4; one launch of 500 steps\n" % cells
                + head + cmds(["trace_tubes", "pmc_tubes_fetch", "pmc_tubes_write", "pmc_copy_fetch",
                               "pmc_copy_write"]) + tail + calib
                + "# the bench's 2-step warm-up launch is also traced; the figures below are the 500-step launch\n"
                + "kernel: %s\ntubes: 512\ncells: %d\nsteps_per_launch: 500\nlaunch_ms: %.3f\n" % (kern, cells, ms)
                + "read_bytes_per_launch: %d\nwrite_bytes_per_launch: %d\ntraffic_bytes_per_launch: %d\n"
                  % (rb, wb, rb + wb)
                + "algorithmic_bytes_per_launch: %d\n" % alg
                + "read_over_algorithmic: %.4f\nwrite_over_algorithmic: %.4f\n" % (2 * rb / alg, 2 * wb / alg)
                + "achieved_algorithmic_GBps: %.1f\n" % (alg / (ms * 1e-3) / 1e9)
                + "source_sha256: %s\n" % digest)
        path = os.path.join(REPO, "profiles", stem + ".txt")
        with open(path, "w") as fh:
            fh.write(text)
        written.append(path)
    return written


def profiled_traffic(kernel, edge):
    """Measured HBM bytes per launch of `kernel` at edge^3 from a committed
    rocprofv3 summary, if that summary was taken of the current sources."""
    from paper_1301_3423_amd.build import source_digest
    prof_dir = os.path.join(REPO, "profiles")
    if not os.path.isdir(prof_dir):
        return None
    digest = source_digest()
    for name in sorted(os.listdir(prof_dir)):
        if not name.endswith(".txt"):
            continue
        kv = {}
        for line in open(os.path.join(prof_dir, name)):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if (kv.get("kernel") == kernel and kv.get("edge") == str(edge)
                and kv.get("source_sha256") == digest and "traffic_bytes_per_launch" in kv):
            return float(kv["traffic_bytes_per_launch"])
    return None


def profile_fields(kernel):
    """The key/value lines of the committed rocprofv3 summary of `kernel`
    (the first one found), if it was taken of the current sources."""
    from paper_1301_3423_amd.build import source_digest
    prof_dir = os.path.join(REPO, "profiles")
    if not os.path.isdir(prof_dir):
        return None
    digest = source_digest()
    for name in sorted(os.listdir(prof_dir)):
        if not name.endswith(".txt"):
            continue
        kv = {}
        for line in open(os.path.join(prof_dir, name)):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel") == kernel and kv.get("source_sha256") == digest:
            return kv
    return None


def time_steps(solver, steps, warmup):
    """Average per-step time (ms) from HIP events on the solver's stream."""
    import torch
    st = solver.stream
    solver.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    solver.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def run_box(edge, precision, fields, steps, warmup, eta_s, order=3, solid=None, pattern="ab"):
    from paper_1301_3423_amd import rlb
    s = rlb.Solver(edge, edge, edge, precision=precision, eta_s=eta_s, order=order, pattern=pattern)
    if solid is not None:
        s.set_walls(solid)
    s.init_fields(*fields)
    c0 = s.conserved()
    ms, wall = time_steps(s, steps, warmup)
    c1 = s.conserved()
    flags, t = s.status()
    read = s.read_fields()
    cells = edge ** 3
    b = 8 if precision == "fp64" else 4
    bytes_per_launch = 2 * Q_OF_ORDER[order] * b * cells
    out = dict(ms_per_step=ms, mlups=cells / (ms * 1e-3) / 1e6, wall_s=wall, flags=flags,
               achieved_gbs=bytes_per_launch / (ms * 1e-3) / 1e9, bytes_per_launch=bytes_per_launch,
               fields=read, t=t, conservation_drift=float(np.max(np.abs(c1 - c0)) / abs(c0[1])),
               conservation_drift_N0=float(abs(c1[0] - c0[0]) / abs(c0[0])))
    del s
    return out


def run_largest_aa(precision, steps, warmup, vmax, eta_s, frac=0.92):
    """The largest box of this precision one GPU holds with the AA pattern
    (edge a multiple of 64, within the library's size cap), fields generated
    on the device."""
    import gc
    import torch
    from paper_1301_3423_amd import inputs, rlb
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    per_cell = rlb.state_bytes(64, 64, 64, precision, 3, "aa") / 64 ** 3 + 40
    edge = int((frac * free / per_cell) ** (1.0 / 3.0)) // 64 * 64
    while edge > 64 and rlb.state_bytes(edge, edge, edge, precision, 3, "aa") == 0:
        edge -= 64
    fields, _ = inputs.random_box_device(edge, edge, edge, vmax, 3)
    torch.cuda.empty_cache()
    s = rlb.Solver(edge, edge, edge, precision=precision, eta_s=eta_s, pattern="aa")
    s.init_fields(*fields)
    s.release_inputs()
    del fields
    torch.cuda.empty_cache()
    c0 = s.conserved()
    ms, wall = time_steps(s, steps, warmup)
    c1 = s.conserved()
    flags, t = s.status()
    cells = edge ** 3
    b = 8 if precision == "fp64" else 4
    out = dict(edge=edge, cells=cells, value=round(cells / (ms * 1e-3) / 1e6, 2), unit="MLUPS",
               ms_per_step=round(ms, 4), achieved_GBps=round(2 * 128 * b * cells / (ms * 1e-3) / 1e9, 1),
               state_GB=round(rlb.state_bytes(edge, edge, edge, precision, 3, "aa") / 1e9, 1),
               two_buffer_GB=round(rlb.state_bytes(edge, edge, edge, precision, 3, "ab") / 1e9, 1),
               gpu_GB=round(total / 1e9, 1), steps=steps, status_flags=flags,
               conservation_drift=float(np.max(np.abs(c1 - c0)) / abs(c0[1])))
    del s
    gc.collect()
    torch.cuda.empty_cache()
    return out


def run_long(edge, precision, fields, steps, eta_s):
    """`steps` steps from the given host fields; fields, status and
    conservation drift at the end, with the wall time of the upload (host
    checks and copies, `init_s`) and of the steps plus the read back to the
    host (`wall_s`)."""
    import torch
    from paper_1301_3423_amd import rlb
    s = rlb.Solver(edge, edge, edge, precision=precision, eta_s=eta_s)
    torch.cuda.synchronize()
    ti = time.perf_counter()
    s.init_fields(*fields)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - ti
    c0 = s.conserved()
    t0 = time.perf_counter()
    s.step(steps)
    out = s.read_fields()
    wall = time.perf_counter() - t0
    c1 = s.conserved()
    flags, t = s.status()
    del s
    return dict(fields=out, flags=flags, t=t, wall_s=wall, init_s=init_s,
                drift=[float(v) for v in (c1 - c0) / np.abs(c0[[0, 1, 1, 1, 1]])])


def field_error_summary(a, b):
    """Max-norm relative error per field; the 4-velocity is compared as a
    4-vector (all components against max |U^mu|), as in the parity tests."""
    out = {}
    for k in ("n", "eps", "P"):
        out[k] = float(np.max(np.abs(a[k] - b[k])) / np.max(np.abs(b[k])))
    us = float(np.max(np.abs(b["U"])))
    for j in range(4):
        out["U%d" % j] = float(np.max(np.abs(a["U"][j] - b["U"][j])) / us)
    return {k: float("%.3e" % v) for k, v in out.items()}


def run_tubes(precision, ntubes=512, steps=500, seed=4):
    """Many independent shock tubes in one persistent launch."""
    import torch
    from paper_1301_3423_amd import inputs, rlb
    spec = inputs.tube_batch(ntubes, seed)
    tubes = [dict(n=t["N"], eta_s=t["eta_s"]) for t in spec]
    b = rlb.Batch(tubes, precision=precision)
    for j, t in enumerate(spec):
        b.init_tube(j, *inputs.shock_tube(t["N"], t["T_left"], t["T_right"]))
    b.step(2)                       # warm-up launch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    lu = sum(t["N"] for t in spec) * steps
    flags = [b.status(j)[0] for j in range(len(spec))]
    bpl = 2 * Q_OF_ORDER[3] * (8 if precision == "fp64" else 4)
    fields = [b.read_tube(j) for j in range(len(spec))]
    return dict(mlups=lu / (ms * 1e-3) / 1e6, ms=ms, cells=sum(t["N"] for t in spec),
                achieved_gbs=lu * bpl / (ms * 1e-3) / 1e9, tubes_flagged=sum(1 for f in flags if f),
                flags=flags, fields=fields)


def latency_stats(lat):
    lat = np.asarray(lat if len(lat) else [0.0])
    return {"p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
            "count": int(len(lat))}


def poisson_stream(sv, reqs, fields, rate, seed, label):
    """Submits reqs at Poisson arrivals of `rate` per second to server sv and
    waits for all of them; returns (completions in id order, makespan s)."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
    done = []
    ids = []

    def keep(cs):   # latency only: the output fields are dropped as they arrive
        done.extend({k: v for k, v in c.items() if k != "fields"} for c in cs)

    start = time.perf_counter()
    for k, (r, f) in enumerate(zip(reqs, fields)):
        while True:
            now = time.perf_counter() - start
            if now >= arrivals[k]:
                break
            keep(sv.poll(wait_ms=max(1, int(1000 * min(arrivals[k] - now, 0.05)))))
        ids.append(sv.submit(r["kind"], r["shape"], r["precision"], r["steps"], f, eta_s=r["eta_s"], outputs=True))
        if (k + 1) % 200 == 0:
            print("bench: serving %s: %d submitted, %d done" % (label, k + 1, len(done)), file=sys.stderr, flush=True)
    keep(sv.drain(timeout_s=900))
    makespan = time.perf_counter() - start
    by_id = {c["id"]: c for c in done}
    return [by_id[i] for i in ids], makespan


def run_serving(nreq, load=0.7, chunk=50, pool_gib=48, seed=5, single_precision_requests=400):
    """Continuous batching under Poisson arrivals: capacity from a saturated
    burst, then nreq requests at rate load * capacity; then the first
    single_precision_requests requests of the same stream again at the same
    rate, once all in float64 and once all in mixed precision."""
    import torch
    from paper_1301_3423_amd import inputs, rlb
    torch.cuda.empty_cache()
    reqs = inputs.serve_requests(nreq, seed)
    cache = {}
    t0 = time.perf_counter()
    fields = [inputs.request_fields(r, cache) for r in reqs]
    print("bench: serving: %d requests generated in %.1f s" % (nreq, time.perf_counter() - t0),
          file=sys.stderr, flush=True)

    def submit(sv, r, f):
        return sv.submit(r["kind"], r["shape"], r["precision"], r["steps"], f, eta_s=r["eta_s"], outputs=True)

    # capacity: a burst of the first requests, all submitted at once.  The
    # same server then takes the Poisson stream: a second server would get
    # new streams, which HIP may map onto hardware queues already shared.
    nburst = min(120, nreq)
    sv = rlb.Server(int(pool_gib) << 30, chunk_steps=chunk, max_tubes=2048)
    tb = time.perf_counter()
    for r, f in zip(reqs[:nburst], fields[:nburst]):
        submit(sv, r, f)
    done = sv.drain(timeout_s=600)
    burst_s = time.perf_counter() - tb
    _, rounds0 = sv.pending()
    capacity = nburst / burst_s
    rate = load * capacity
    print("bench: serving capacity %.1f solves/s; Poisson rate %.1f/s" % (capacity, rate),
          file=sys.stderr, flush=True)
    # Poisson arrivals
    done, makespan = poisson_stream(sv, reqs, fields, rate, seed + 1, "mix")
    _, rounds = sv.pending()
    rounds -= rounds0
    lat = np.array([c["t_done"] - c["t_submit"] for c in done])
    kinds, precs = {}, {}
    for c, r in zip(done, reqs):
        kinds.setdefault(r["kind"], []).append(c["t_done"] - c["t_submit"])
        precs.setdefault(r["precision"], []).append(c["t_done"] - c["t_submit"])
    out = {
        "workload": "%d requests, Poisson arrivals at %.2f x measured capacity; 70%% tubes (N 200-8000, "
                    "100-2000 steps), 30%% boxes (32^3-128^3, |v|<=0.6, 200-1000 steps), eta/s U(0.01,0.5), "
                    "FP64/mixed 50/50" % (nreq, load),
        "capacity_solves_per_s": round(capacity, 2), "arrival_rate_per_s": round(rate, 2),
        "solves_per_s": round(len(done) / makespan, 2),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "p50_tube_s": round(float(np.percentile(kinds.get("tube", [0]), 50)), 4),
        "p50_box_s": round(float(np.percentile(kinds.get("box", [0]), 50)), 4),
        "p99_tube_s": round(float(np.percentile(kinds.get("tube", [0]), 99)), 4),
        "p99_box_s": round(float(np.percentile(kinds.get("box", [0]), 99)), 4),
        "by_precision": {p: latency_stats(v) for p, v in sorted(precs.items())},
        "flagged": int(sum(1 for c in done if c["flags"])), "errors": int(sum(1 for c in done if c["rc"])),
        "rounds": int(rounds), "chunk_steps": chunk, "completed": len(done),
    }
    # the same requests, all in one precision, at the same arrival rate
    m = min(single_precision_requests, nreq)
    if m > 0:
        single = {}
        for prec in ("fp64", "mixed"):
            rq = [dict(r, precision=prec) for r in reqs[:m]]
            d, span = poisson_stream(sv, rq, fields[:m], rate, seed + 2, prec)
            lat1 = [c["t_done"] - c["t_submit"] for c in d]
            single[prec] = dict(latency_stats(lat1), solves_per_s=round(len(d) / span, 2),
                                p99_tube_s=latency_stats([x for x, r in zip(lat1, rq) if r["kind"] == "tube"])["p99_s"],
                                p99_box_s=latency_stats([x for x, r in zip(lat1, rq) if r["kind"] == "box"])["p99_s"],
                                errors=int(sum(1 for c in d if c["rc"])))
        out["single_precision_streams"] = dict(
            workload="the first %d requests of the stream, all float64 or all mixed precision, Poisson arrivals "
                     "at the same rate (%.2f/s, same arrival seed for both)" % (m, rate), **single)
    sv.close()
    return out


def run_riemann():
    """Latency of the 1D Riemann problems: the 1x1x200 tube (T 1.0 | 0.8,
    eta/s 0.1, 200 steps, FP64) and the paper's 1x1x1600 tube (T 1.0 | 0.5,
    eta/s 0.5 and 0.1, t = 3.2 fm/c: 63 steps of the third-order model, 133
    of the second-order one), each as one persistent launch, wall time from
    submission of the launch to fields on the host; and the largest
    difference between the two models' velocity profiles."""
    import torch
    from paper_1301_3423_amd import inputs, rlb
    out = {}
    profiles = {}
    for name, n, tl, tr, es, steps, order in (("tube_200", 200, 1.0, 0.8, 0.1, 200, 3),
                                              ("paper_1600", 1600, 1.0, 0.5, 0.5, 63, 3),
                                              ("paper_1600_eta0.1", 1600, 1.0, 0.5, 0.1, 63, 3),
                                              ("paper_1600_order2", 1600, 1.0, 0.5, 0.5, 133, 2),
                                              ("paper_1600_order2_eta0.1", 1600, 1.0, 0.5, 0.1, 133, 2)):
        b = rlb.Batch([dict(n=n, eta_s=es)], precision="fp64", order=order)
        f = inputs.shock_tube(n, tl, tr)
        b.init_tube(0, *f)
        b.step(2)
        b.init_tube(0, *f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        r = b.read_tube(0)
        dt = time.perf_counter() - t0
        vz = r["U"][3] / r["U"][0]
        profiles[name] = vz
        out[name] = {"cells": n, "steps": steps, "order": order, "eta_s": es, "wall_ms": round(dt * 1e3, 3),
                     "max_vz": round(float(np.max(np.abs(vz))), 4), "flags": b.status(0)[0]}
    # the paper's second- vs third-order comparison at t = 3.2 fm/c (Figs. 4-5)
    out["max_abs_dvz_3rd_vs_2nd"] = {
        "eta_s_0.1": round(float(np.max(np.abs(profiles["paper_1600_eta0.1"] - profiles["paper_1600_order2_eta0.1"]))), 4),
        "eta_s_0.5": round(float(np.max(np.abs(profiles["paper_1600"] - profiles["paper_1600_order2"]))), 4)}
    return out


def roofline(r, kernel, edge):
    return {"bound": "hbm", "achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(kernel, edge),
            "kernel": kernel, "algorithmic_bytes_per_launch": r["bytes_per_launch"]}


def _oracle_box_worker(job):
    """One oracle run on its own box (a separate process, one thread):
    returns (lattice updates, seconds)."""
    edge, steps, vmax, eta_s, seed = job
    from threadpoolctl import threadpool_limits
    import oracle
    from oracle import rlb as orlb
    from paper_1301_3423_amd import inputs
    with threadpool_limits(limits=1):
        o = orlb.Solver(edge, edge, edge, lat=oracle.load_lattice(), eta_s=eta_s)
        o.init_fields(*inputs.random_box(edge, edge, edge, vmax, seed=seed))
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
    return edge ** 3 * steps, dt


# host cores given to the CPU baseline's parallel leg: the CPU share of one
# GPU on a shared node (os.cpu_count() may report the whole machine)
CPU_WORKERS = 16


def cpu_baseline(vmax, eta_s):
    """The FP64 oracle on a bounded sample of the same workload: one process
    per host core, each stepping its own box of the same recipe (the oracle
    is single-threaded array code; boxes are independent), timed over the
    parallel region; plus the one-core figure of a single process."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    lu1, dt1 = _oracle_box_worker((64, 10, vmax, eta_s, 3))
    workers = max(1, min(CPU_WORKERS, os.cpu_count() or 1))
    edge, steps = 48, 6
    jobs = [(edge, steps, vmax, eta_s, 100 + k) for k in range(workers)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_box_worker, [(8, 1, vmax, eta_s, 1)] * workers))   # start the interpreters
        t0 = time.perf_counter()
        res = list(ex.map(_oracle_box_worker, jobs))
        wall = time.perf_counter() - t0
    lu = sum(r[0] for r in res)
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=lu / wall / 1e6, unit="MLUPS", cores=workers, kind="oracle",
                sample="%d processes, each the numpy FP64 oracle (one thread) on its own %d^3 box of the same "
                       "field generator (v_max %.2g, eta/s %.2g, seeds 100..%d), %d steps; aggregate lattice "
                       "updates over the wall time of the parallel region (%.1f s) on %s, %d CPUs visible"
                       % (workers, edge, vmax, eta_s, 99 + workers, steps, wall, cpu, os.cpu_count() or 0),
                single_thread={"value": lu1 / dt1 / 1e6, "unit": "MLUPS", "cores": 1,
                               "sample": "one process, 64^3 box (seed 3), 10 steps, %.1f s" % dt1})


def main():
    args = parse()
    if args.summarize_profiles:
        for path in summarize_profiles(args.summarize_profiles):
            print(path)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1301_3423_amd import inputs
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    edge = args.edge
    copy_gbs = copy_bandwidth()
    print("bench: plain copy %.0f GB/s" % copy_gbs, file=sys.stderr, flush=True)
    ceiling = stream_ceiling()
    print("bench: streaming kernels: copy %.0f GB/s, read %.0f GB/s, write %.0f GB/s"
          % (ceiling["copy_GBps"], ceiling["read_GBps"], ceiling["write_GBps"]), file=sys.stderr, flush=True)
    print("bench: generating %d^3 fields" % edge, file=sys.stderr, flush=True)
    fields = inputs.random_box(edge, edge, edge, args.vmax, seed=3)
    print("bench: mixed precision", file=sys.stderr, flush=True)
    mixed = run_box(edge, "mixed", fields, args.steps, args.warmup, args.eta_s)
    print("bench: mixed %.1f MLUPS" % mixed["mlups"], file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_box(edge, "fp64", fields, args.steps, args.warmup, args.eta_s)
        print("bench: fp64 %.1f MLUPS" % fp64["mlups"], file=sys.stderr, flush=True)
    second = {}
    if not args.no_second_order:
        for prec in ("mixed", "fp64"):
            if prec == "fp64" and args.no_fp64:
                continue
            r = run_box(edge, prec, fields, args.steps, args.warmup, args.eta_s, order=2)
            print("bench: second-order %s %.1f MLUPS" % (prec, r["mlups"]), file=sys.stderr, flush=True)
            second[prec] = {"value": round(r["mlups"], 2), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 4),
                            "roofline": roofline(r, kernel_name(2, prec, edge), edge),
                            "status_flags": r["flags"], "conservation_drift": r["conservation_drift"]}
    walls = None
    if not args.no_walls:
        # a channel: solid slabs of 6 cells (the largest displacement) at both y ends
        solid = np.zeros((edge, edge, edge), dtype=bool)
        solid[:, :6, :] = True
        solid[:, -6:, :] = True
        fluid = int((~solid).sum())
        r = run_box(edge, "mixed", fields, args.steps, args.warmup, args.eta_s, solid=solid)
        print("bench: walls mixed %.1f MLUPS" % r["mlups"], file=sys.stderr, flush=True)
        walls = {"workload": "the same %d^3 box as a channel: solid slabs of 6 cells at both y ends (%.1f%% "
                             "solid), link-wise bounce-back, mixed precision, third order"
                             % (edge, 100.0 * (1 - fluid / edge ** 3)),
                 "value": round(r["mlups"], 2), "unit": "MLUPS (all cells)",
                 "fluid_mlups": round(r["mlups"] * fluid / edge ** 3, 2), "ms_per_step": round(r["ms_per_step"], 4),
                 "vs_periodic": round(r["ms_per_step"] / mixed["ms_per_step"], 3),
                 "status_flags": r["flags"], "N0_drift": r["conservation_drift_N0"]}
    aa = {}
    if not args.no_aa:
        for prec, ab in (("mixed", mixed), ("fp64", fp64)):
            if ab is None:
                continue
            r = run_box(edge, prec, fields, args.steps, args.warmup, args.eta_s, pattern="aa")
            print("bench: AA %s %.1f MLUPS" % (prec, r["mlups"]), file=sys.stderr, flush=True)
            same = all(np.array_equal(r["fields"][k], ab["fields"][k]) for k in ("n", "eps", "P", "U"))
            traffic = {acc: profiled_traffic(kernel_name(3, prec, edge, acc), edge) for acc in ("aa_even", "aa_odd")}
            aa[prec] = {"value": round(r["mlups"], 2), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 4),
                        "vs_ab": round(ab["ms_per_step"] / r["ms_per_step"], 3),
                        "achieved_GBps": round(r["achieved_gbs"], 1), "fields_equal_ab": bool(same),
                        "traffic_bytes_per_launch": traffic,
                        "status_flags": r["flags"], "conservation_drift": r["conservation_drift"]}
    largest = None
    if not args.no_aa and not args.no_fp64 and not args.no_largest:
        largest = run_largest_aa("fp64", min(args.steps, 20), 2, args.vmax, args.eta_s)
        print("bench: largest AA fp64 box %d^3: %.1f MLUPS" % (largest["edge"], largest["value"]),
              file=sys.stderr, flush=True)
    configs = {}
    if not args.no_configs and not args.no_fp64:
        from paper_1301_3423_amd import inputs as _inp
        f2 = _inp.random_box(128, 128, 128, 0.5, seed=2)
        r = run_long(128, "fp64", f2, 1000, 0.2)
        configs["box_128cube_fp64_1000_steps"] = {
            "workload": "128^3 periodic box, float64, |v|<=0.5, T=1+-10%, eta/s=0.2 (seed 2), 1000 steps",
            "mlups": round(128 ** 3 * 1000 / r["wall_s"] / 1e6, 1),
            "mlups_host_inclusive": round(128 ** 3 * 1000 / (r["init_s"] + r["wall_s"]) / 1e6, 1),
            "upload_s": round(r["init_s"], 4), "status_flags": r["flags"],
            "drift_N0_T00_T0x_T0y_T0z": r["drift"],
            "note": "drift = (final - initial) / |initial| for N^0 and T^00, and relative to T^00 for the "
                    "momenta; mlups from the wall clock of the steps and the read back to the host, "
                    "mlups_host_inclusive with the upload of the host fields (upload_s) added"}
        del f2
        print("bench: 128^3 fp64 1000 steps done", file=sys.stderr, flush=True)
        rm = run_long(edge, "mixed", fields, 2000, args.eta_s)
        rd = run_long(edge, "fp64", fields, 2000, args.eta_s)
        configs["box_%dcube_mixed_vs_fp64_2000_steps" % edge] = {
            "workload": "the %d^3 benchmark box, 2000 steps in each precision" % edge,
            "max_rel": field_error_summary(rm["fields"], rd["fields"]),
            "status_flags": [rm["flags"], rd["flags"]], "drift_mixed": rm["drift"], "drift_fp64": rd["drift"],
            "mlups_host_inclusive": {
                k: round(edge ** 3 * 2000 / (r["init_s"] + r["wall_s"]) / 1e6, 1) for k, r in (("mixed", rm), ("fp64", rd))},
            "upload_s": {k: round(r["init_s"], 4) for k, r in (("mixed", rm), ("fp64", rd))},
            "read_back_s_plus_steps_s": {k: round(r["wall_s"], 4) for k, r in (("mixed", rm), ("fp64", rd))},
            "note": "max-norm relative error of the mixed path against the float64 GPU path (pinned to the "
                    "oracle at this size on sampled cells); mlups_host_inclusive runs from host fields to "
                    "host fields (upload with its host checks, 2000 steps, read back), while the headline "
                    "value starts and ends with the state resident in HBM"}
        del rm, rd
        print("bench: %d^3 2000-step comparison done" % edge, file=sys.stderr, flush=True)
    tubes = {}
    tube_runs = {}
    if not args.no_tubes:
        for prec in ("fp64", "mixed"):
            r = run_tubes(prec)
            tube_runs[prec] = r
            print("bench: tubes %s %.1f MLUPS" % (prec, r["mlups"]), file=sys.stderr, flush=True)
            kv = profile_fields("k_tubes<Model<3>, %s>" % ("double" if prec == "fp64" else "float")) or {}
            tubes[prec] = {"value": round(r["mlups"], 2), "unit": "MLUPS", "launch_ms": round(r["ms"], 3),
                           "achieved_GBps": round(r["achieved_gbs"], 1), "cells": r["cells"],
                           "tubes_flagged": r["tubes_flagged"],
                           "profiled_read_over_algorithmic": float(kv["read_over_algorithmic"])
                           if "read_over_algorithmic" in kv else None,
                           "profiled_write_over_algorithmic": float(kv["write_over_algorithmic"])
                           if "write_over_algorithmic" in kv else None}
    riemann = run_riemann()
    serving = None
    if args.serve_requests > 0:
        serving = run_serving(args.serve_requests)
        print("bench: serving p50 %.3f s p99 %.3f s, %.1f solves/s" % (
            serving["p50_latency_s"], serving["p99_latency_s"], serving["solves_per_s"]), file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_baseline(args.vmax, args.eta_s)
    mixed_kernel = kernel_name(3, "mixed", edge)
    line = {
        "metric": "MLUPS at 256^3 FP64 vs FP32-mixed (% HBM roofline); served p50/p99 latency",
        "value": round(mixed["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "3D periodic box %d^3, mixed precision (float32 populations, float64 "
                               "moments/Landau frame), random fields |v|<=%.2g, T=1+-10%%, eta/s=%.2g%s"
                               % (edge, args.vmax, args.eta_s, VMAX_NOTE if args.vmax == 0.6 else ""),
                   "cells": edge ** 3, "parallelism": "single GPU"},
        "roofline": roofline(mixed, mixed_kernel, edge),
        "status_flags": mixed["flags"],
        "conservation_drift": mixed["conservation_drift"],
        "copy_GBps": round(copy_gbs, 1),
        "stream_ceiling": ceiling,
    }
    best_copy = max(ceiling["copy_GBps"], ceiling["copy_nontemporal_GBps"])
    ceiling["mixed_step_over_best_copy"] = round(line["roofline"]["achieved"] / best_copy, 3)
    if fp64 is not None:
        line["fp64"] = {"value": round(fp64["mlups"], 2), "unit": "MLUPS", "dtype": "f64",
                        "ms_per_step": round(fp64["ms_per_step"], 4),
                        "roofline": roofline(fp64, kernel_name(3, "fp64", edge), edge),
                        "status_flags": fp64["flags"],
                        "conservation_drift": fp64["conservation_drift"],
                        "mixed_over_fp64": round(mixed["mlups"] / fp64["mlups"], 3)}
        # both runs start from the same fields and take the same steps
        line["mixed_vs_fp64_error"] = {
            "steps": mixed["t"],
            "max_rel": field_error_summary(mixed["fields"], fp64["fields"]),
            "note": "max-norm relative error of the mixed path against the float64 GPU path at 256^3 "
                    "(the float64 path is pinned to the oracle at these sizes on sampled cells)"}
    if second:
        line["second_order"] = {"workload": "the same %d^3 box and fields with the second-order model of "
                                            "Appendix A (66 points, R = 3)" % edge, **second}
    if walls is not None:
        line["walls"] = walls
    if aa:
        line["aa_pattern"] = {"workload": "the same %d^3 box, fields and steps, third order, one population "
                                          "buffer updated in place (AA pattern) instead of two" % edge, **aa}
    if largest is not None:
        line["aa_largest_fp64"] = {
            "workload": "the largest float64 third-order box this GPU holds with the AA pattern (%d^3, random "
                        "fields generated on the device, same recipe); the two-buffer layout would need "
                        "%.0f GB" % (largest["edge"], largest["two_buffer_GB"]), **largest}
    if configs:
        line["full_length_runs"] = configs
    if tubes:
        line["tubes"] = {"workload": "512 shock tubes 1x1xN, N~U{200..4000}, T_L/T_R~U(1.1,2), "
                                     "eta/s in {0.01,0.05,0.1,0.2,0.5}, 500 steps, one persistent launch",
                         **tubes}
        if len(tube_runs) == 2:
            a, b = tube_runs["mixed"], tube_runs["fp64"]
            errs = [max(field_error_summary(fa, fb).values())
                    for fa, fb, ga, gb in zip(a["fields"], b["fields"], a["flags"], b["flags"]) if not (ga or gb)]
            line["tubes"]["per_tube_error_mixed_vs_fp64"] = {
                "tubes": len(errs), "max": float("%.3e" % max(errs)), "median": float("%.3e" % np.median(errs)),
                "note": "max-norm relative error over n, eps, U, P of each unflagged tube after 502 steps; the "
                        "float64 tube path is pinned to the oracle in the tests"}
    line["riemann_fp64"] = riemann
    if serving is not None:
        line["serving"] = serving
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    # the process ends once the HIP runtime has returned the device memory
    # the legs reserved (hundreds of GB after the largest AA box): release it
    # here, timed, rather than in the interpreter's exit
    t0 = time.perf_counter()
    del mixed, fp64, fields, second, aa, largest, configs, tubes, tube_runs
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print("bench: device memory released in %.2f s; exiting at unix time %.3f"
          % (time.perf_counter() - t0, time.time()), file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
