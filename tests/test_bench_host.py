"""Host logic of bench.py's profile reducers, on synthetic rocprofv3 CSV
traces (no GPU)."""
import csv
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def write_trace(path, dispatches):
    rows, t = [], 0
    for i, (name, dur, gap) in enumerate(dispatches):
        rows.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + dur})
        t += dur + gap
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_batch_trace_summary(tmp_path):
    steps, warmup = 3, 1
    d = []
    for _ in range(3 * (steps + warmup)):          # persistent kernel, three variants
        d += [("fft_pass_kernel<tuner>", 1_000, 100), ("offt::many_kernel_batch_f32(offt::ManyArgs)", 900_000, 100)]
    for v in range(2):                               # level kernels, direct then graph
        for _ in range(steps + warmup):
            d += [("offt::many_level_kernel_batch_f32(offt::ManyArgs, long)", 100_000 * (k + 1), 2_000 * v)
                  for k in range(3)]
    for _ in range(2 * (steps + warmup)):
        d.append(("offt::many_sync_kernel_batch_f32(offt::ManyArgs, offt::ManySyncArgs)", 700_000, 100))
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    txt = load_bench().summarize_batch(str(tmp_path), "cmd", steps, warmup)
    rows = {l[:38].strip(): l[38:].split() for l in txt.splitlines() if not l.startswith("#")}
    assert rows["persistent work-queue kernel"] == ["12", "900.00", "1.00", "900.00"]
    assert rows["level kernels"] == ["24", "200.00", "3.00", "600.00"]
    assert rows["level-synchronous persistent kernel"] == ["8", "700.00", "1.00", "700.00"]
    # graph replays: 3 kernels of 100, 200 and 300 us with 2 us between them
    replay = [l for l in txt.splitlines() if "graph replays" in l][0]
    assert "3 level kernels per execution" in replay
    assert "span first start to last end 604.00 us" in replay and "summed kernel time 600.00 us" in replay
