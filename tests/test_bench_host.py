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
    runs = steps + warmup
    d = []
    for _ in range(3 * runs):                        # persistent kernel, three variants
        d += [("fft_pass_kernel<tuner>", 1_000, 100), ("offt::many_kernel_batch_f32(offt::ManyArgs)", 900_000, 100)]
    lvl = "offt::many_level_kernel_batch_f32(offt::ManyArgs, long)"
    for v in range(2):                               # level kernels, direct then graph
        for _ in range(runs):
            d += [(lvl, 100_000 * (k + 1), 2_000 * v) for k in range(3)]
    for _ in range(runs):                            # grouped graph: 2 groups of 3 levels
        d += [(lvl, 50_000, 1_000) for _ in range(6)]
    for _ in range(2 * runs):
        d.append(("offt::many_sync_kernel_batch_f32(offt::ManyArgs, offt::ManySyncArgs)", 700_000, 100))
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    txt = load_bench().summarize_batch(str(tmp_path), "cmd", steps, warmup)
    rows = {l[:46].strip(): l[46:].split() for l in txt.splitlines() if not l.startswith(("#", " "))}
    assert rows["persistent work-queue kernel"] == ["12", "900.00", "1.00", "900.00"]
    assert rows["level kernels, direct"] == ["12", "200.00", "3.00", "600.00"]
    assert rows["level kernels, graph"] == ["12", "200.00", "3.00", "600.00"]
    assert rows["level kernels, grouped graph"] == ["24", "50.00", "6.00", "300.00"]
    assert rows["level-synchronous persistent kernel"] == ["8", "700.00", "1.00", "700.00"]
    assert rows["every-length executor, level kernels, direct"] == ["none", "traced"]
    replays = [l for l in txt.splitlines() if "graph replays" in l]
    # level graph: 3 kernels of 100, 200 and 300 us with 2 us between them
    assert "3 kernels per execution" in replays[0]
    assert "span first start to last end 604.00 us" in replays[0] and "summed kernel time 600.00 us" in replays[0]
    # grouped graph: 6 kernels of 50 us with 1 us between them
    assert "6 kernels per execution" in replays[1] and "span first start to last end 305.00 us" in replays[1]


def test_nd_trace_summary(tmp_path):
    steps, warmup = 2, 1
    res = [{"shape": [8, 8, 8, 8], "dtype": "f32",
            "tuned": {"ms": 0.01, "plan": "order=dacb;a=8/8;b=8/8;c=8/8/x;d=8/8"},
            "heuristic": {"ms": 0.02, "plan": "order=dcba;a=8/8/x;b=8/8/x;c=8/8/x;d=8/8"}}]
    log = tmp_path / "nd.log"
    log.write_text("noise\n" + __import__("json").dumps({"nd": res}) + "\n")
    d = []
    for plan_scale in (1, 2):
        for st in range(warmup + steps):
            # warm-up transforms take 50 us per pass, so a wrong split shows in the means
            d += [("twiddle_kernel", 5, 0)] if st == 0 else []
            d += [("offt::fft_pass_kernel<...>", (50_000 if st < warmup else 1_000 * (i + 1) * plan_scale), 10)
                  for i in range(4)]
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    txt = load_bench().summarize_nd(str(tmp_path), str(log), "cmd", steps, warmup)
    passes = [l.split() for l in txt.splitlines() if l.startswith("  pass")]
    assert [p[2] for p in passes[:4]] == ["d=8/8", "a=8/8", "c=8/8/x", "b=8/8"]
    assert [float(p[3]) for p in passes] == [1.0, 2.0, 3.0, 4.0, 2.0, 4.0, 6.0, 8.0]
    # 2 * 4096 points * 8 bytes in 1 us = 65.5 GB/s
    assert float(passes[0][5]) == 65.5
    assert "summed pass time 10.0 us" in txt and "summed pass time 20.0 us" in txt


def test_nd_trace_summary_with_slab_schedule(tmp_path):
    """A 4-axis slab schedule: the pass over a once, then b, c, d once per
    slab (8 planes in slabs of 3: three slabs)."""
    b = load_bench()
    steps, warmup = 2, 1
    plan = "order=adcb;a=8/8;b=8/8;c=8/8;d=8/8;slab=3"
    res = [{"shape": [8, 8, 8, 8], "dtype": "f32", "tuned": {"ms": 0.01, "plan": plan},
            "heuristic": {"ms": 0.02, "plan": "order=dcba;a=8/8;b=8/8;c=8/8;d=8/8"}}]
    log = tmp_path / "nd.log"
    log.write_text(__import__("json").dumps({"nd": res}) + "\n")
    d = []
    for p in (plan, res[0]["heuristic"]["plan"]):
        for st in range(warmup + steps):
            d += [("offt::fft_pass_kernel<...>", 50_000 if st < warmup else (100 * (i + 1) if b.plan_slab(p) and i
                                                                            else 1_000), 10)
                  for i in b.pass_launches(p, 8)]
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    txt = b.summarize_nd(str(tmp_path), str(log), "cmd", steps, warmup)
    passes = [l.split() for l in txt.splitlines() if l.startswith("  pass")]
    assert [p[2] for p in passes[:4]] == ["a=8/8", "d=8/8;slab=3", "c=8/8;slab=3", "b=8/8;slab=3"]
    # three slabs of 0.2, 0.3 and 0.4 us per pass
    assert [float(p[3]) for p in passes[:4]] == [1.0, 0.6, 0.9, 1.2]
    assert [float(p[3]) for p in passes[4:]] == [1.0, 1.0, 1.0, 1.0]


def test_reversed_trace_summary(tmp_path):
    steps, warmup, n = 2, 1, 8
    nat = "order=bca;a=8/8;b=8/8/x;c=8/8"
    rev = "order=cba;rev=a;a=8/8;b=8/8/x;c=8/8|order=bca;rev=a;a=8/8;b=8/8;c=8/8"
    res = {"workload": "w"}
    for dt in ("f64", "f32"):
        res[dt] = {"natural": {"fwd_ms": 0.006, "bwd_ms": 0.006, "plan": nat},
                   "reversed": {"fwd_ms": 0.007, "bwd_ms": 0.008, "plan": rev}}
    log = tmp_path / "rev.log"
    log.write_text(__import__("json").dumps({"reversed_output": res}) + "\n")
    d = []
    for run in range(8):                 # (f64, f32) x (natural, reversed) x (fwd, bwd)
        for st in range(warmup + steps):
            for i in range(3):
                name = "offt::fft_tpass_kernel<...>" if run % 4 >= 2 and i == 2 - (run % 2) else \
                    "offt::fft_pass_kernel<...>"
                d.append((name, 99_000 if st < warmup else 1_000 * (run + 1) + 100 * i, 10))
            d.append(("offt::fill_uniform_kernel", 7, 0))
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    txt = load_bench().summarize_reversed(str(tmp_path), str(log), "cmd", n, steps, warmup)
    passes = [l.split() for l in txt.splitlines() if l.startswith("  pass")]
    assert len(passes) == 24
    assert [p[2] for p in passes[6:9]] == ["c=8/8", "b=8/8/x", "a=8/8"]
    assert passes[8][3] == "(T)" and passes[9][2] == "b=8/8" and passes[10][2] == "c=8/8"
    assert passes[11][2] == "a=8/8" and passes[11][3] == "(T)"
    assert [float(p[-4]) for p in passes[:3]] == [1.0, 1.1, 1.2]
    assert float(passes[23][-4]) == 8.2


def test_reversed_trace_summary_with_slab_natural_plan(tmp_path):
    """The natural plan beside the reversed one may run a slab schedule: its
    later passes are summed over their slabs."""
    b = load_bench()
    steps, warmup, n = 2, 1, 8
    nat = "order=acb;a=8/8;b=8/8/x;c=8/8;slab=4"
    rev = "order=cba;rev=a;a=8/8;b=8/8/x;c=8/8|order=bca;rev=a;a=8/8;b=8/8;c=8/8"
    res = {"workload": "w"}
    for dt in ("f64", "f32"):
        res[dt] = {"natural": {"fwd_ms": 0.006, "bwd_ms": 0.006, "plan": nat},
                   "reversed": {"fwd_ms": 0.007, "bwd_ms": 0.008, "plan": rev}}
    log = tmp_path / "rev.log"
    log.write_text(__import__("json").dumps({"reversed_output": res}) + "\n")
    d = []
    for run in range(8):
        plan = nat if run % 4 < 2 else rev.split("|")[run % 2]
        for st in range(warmup + steps):
            for i in b.pass_launches(plan, n):
                slabbed = b.plan_slab(plan) and i > 0
                d.append(("offt::fft_pass_kernel<...>", 99_000 if st < warmup else (250 if slabbed else 1_000), 10))
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    txt = b.summarize_reversed(str(tmp_path), str(log), "cmd", n, steps, warmup)
    passes = [l.split() for l in txt.splitlines() if l.startswith("  pass")]
    assert len(passes) == 24
    assert [p[2] for p in passes[:3]] == ["a=8/8", "c=8/8;slab=4", "b=8/8/x;slab=4"]
    # two slabs of 0.25 us per slab pass
    assert [float(p[3]) for p in passes[:3]] == [1.0, 0.5, 0.5]


def test_stats_summary_with_copy_kernels(tmp_path):
    """Per-pass means of a headline run from the dispatch trace: the
    transform's passes, then each pass's copy kernel, per timed plan."""
    steps, warmup, n = 2, 1, 8
    p64, p32 = "order=cba;a=8/8;b=8/8/x;c=8/8", "order=abc;a=8/8;b=8/8;c=8/8"
    log = tmp_path / "stats.log"
    log.write_text("noise\n" + __import__("json").dumps({"plan": p64, "f32": {"plan": p32}}) + "\n")
    d = []
    for scale in (1, 2):                                   # complex128 run, then complex64
        for st in range(warmup + steps):
            d += [("offt::fft_pass_kernel<...>", (90_000 if st < warmup else 1_000 * (i + 1) * scale), 10)
                  for i in range(3)]
        for i in range(3):
            d += [("offt::copy_pattern_kernel<...>", (70_000 if st < warmup else 500 * (i + 1) * scale), 10)
                  for st in range(warmup + steps)]
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    with open(tmp_path / "run" / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs",
                                          "Percentage"])
        w.writeheader()
        w.writerow({"Name": "offt::fft_pass_kernel<...>", "Calls": 18, "TotalDurationNs": 1, "AverageNs": 1,
                    "MinNs": 1, "MaxNs": 1, "Percentage": 100})
    txt = load_bench().summarize_stats(str(tmp_path), str(log), "cmd", n, steps, warmup)
    passes = [l.split() for l in txt.splitlines() if l.startswith("  pass")]
    assert [float(p[4]) for p in passes] == [1.0, 2.0, 3.0, 2.0, 4.0, 6.0]
    # copy kernels at half the pass time: "of copy" 0.5
    assert [float(p[p.index("copy") + 1]) for p in passes] == [0.5, 1.0, 1.5, 1.0, 2.0, 3.0]
    assert all(float(p[p.index("of") + 2]) == 0.5 for p in passes)
    # 2 * 512 points * 16 bytes in 1 us = 16.4 GB/s; the copy in 0.5 us, 32.8
    first = [l for l in txt.splitlines() if l.startswith("  pass")][0]
    assert "16.4 GB/s" in first and "32.8 GB/s" in first


def test_stats_summary_with_slab_schedule(tmp_path):
    """A slab schedule launches its passes once per slab, slab after slab:
    per pass and step the slabs' dispatches are summed."""
    b = load_bench()
    steps, warmup, n = 2, 1, 8
    p64, p32 = "order=abc;a=8/8;b=8/8;c=8/8", "order=abc;a=8/8;b=8/8;c=8/8;slab=3"
    assert b.pass_launches(p32, n) == [0, 1, 2, 1, 2, 1, 2]        # slabs of 3, 3 and 2 planes
    assert b.pass_launches(p64, n) == [0, 1, 2]
    assert b.pass_groups(p32) == [[0], [1, 2]] and b.pass_groups(p64) == [[0], [1], [2]]
    assert b.group_key(p32, [1, 2]) == "b=8/8+c=8/8;slab=3"
    assert b.pass_label(p32, 0) == "a=8/8" and b.pass_label(p32, 2) == "c=8/8;slab=3"
    log = tmp_path / "stats.log"
    log.write_text(__import__("json").dumps({"plan": p64, "f32": {"plan": p32}}) + "\n")
    d = []
    for plan in (p64, p32):
        for st in range(warmup + steps):
            for i in b.pass_launches(plan, n):
                slabbed = b.plan_slab(plan) and i > 0
                d.append(("offt::fft_pass_kernel<...>", 90_000 if st < warmup else (300 if slabbed else 1_000), 10))
        for i in range(3):
            d += [("offt::copy_pattern_kernel<...>", 500, 10) for _ in range(warmup + steps)]
    write_trace(str(tmp_path / "run" / "run_kernel_trace.csv"), d)
    with open(tmp_path / "run" / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs",
                                          "Percentage"])
        w.writeheader()
        w.writerow({"Name": "offt::fft_pass_kernel<...>", "Calls": 30, "TotalDurationNs": 1, "AverageNs": 1,
                    "MinNs": 1, "MaxNs": 1, "Percentage": 100})
    txt = b.summarize_stats(str(tmp_path), str(log), "cmd", n, steps, warmup)
    passes = [l.split() for l in txt.splitlines() if l.startswith("  pass")]
    assert [float(p[4]) for p in passes] == [1.0, 1.0, 1.0, 1.0, 0.9, 0.9]
    assert [p[2] for p in passes][3:] == ["a=8/8", "b=8/8;slab=3", "c=8/8;slab=3"]


def test_roofline_and_copy_ceilings_of_a_slab_schedule():
    b = load_bench()
    res = {"plan": "order=abc;a=8/8;b=8/8;c=8/8;slab=3", "groups": [[0], [1, 2]], "pass_ms": [1.0, 1.5],
           "copy_ms": [0.8, 0.6, 0.6], "pass_bytes": 10 ** 9}
    r = b.roofline(res, "8_f32")
    # the slab group takes longer, but the dominant single-launch kernel is pass a
    assert r["kernel"] == "a=8/8" and r["kernel_ms"] == 1.0 and r["achieved"] == 1000.0
    c = b.copy_ceilings(res)
    assert [x["pass"] for x in c] == ["a=8/8", "b=8/8+c=8/8;slab=3"]
    assert c[1]["copy_ms"] == 1.2 and c[1]["pass_gbs"] == round(2e9 / 1.5e6, 1) and c[1]["frac_of_copy"] == 0.8
