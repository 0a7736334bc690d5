"""Host-side measurement tooling (CPU): the rocprofv3 summarizer and bench.py's
argument contract."""
import json
import os
import subprocess
import sys

from paper_2305_03945_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_trace(path, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for name, s, e in rows:
            f.write('"%s",%d,%d\n' % (name, s, e))


def test_trace_table_averages_and_drops_converged_launches(tmp_path):
    k = "void rdk::k_cols<float, 11, 0, 1, 2>(rdk::Slot* const*)"
    # three working launches of 10, 12, 14 us and one early return of 1 us
    _write_trace(tmp_path / "x_kernel_trace.csv", [(k, 0, 10000), (k, 20000, 32000), (k, 40000, 54000),
                                                   (k, 60000, 61000)])
    t = profsum.trace_table(str(tmp_path / "x_kernel_trace.csv"))
    assert len(t) == 1 and t[0]["kernel"] == "k_cols<float,11,0,1,2>"
    assert t[0]["calls"] == 4 and t[0]["working_calls"] == 3
    assert abs(t[0]["working_avg_us"] - 12.0) < 1e-9
    assert abs(t[0]["avg_us"] - 37.0 / 4) < 1e-9


def test_trace_table_lists_the_outer_updates_of_the_mixed_row_pass_apart(tmp_path):
    k = "void rdk::k_row_forward<float, 11, 0, 0, 5>(rdk::Slot* const*)"
    # five inner launches of 16 us, two outer updates of 40 us, one early return
    rows = [(k, 100000 * i, 100000 * i + 16000) for i in range(5)]
    rows += [(k, 600000, 640000), (k, 700000, 740000), (k, 800000, 801000)]
    _write_trace(tmp_path / "x_kernel_trace.csv", rows)
    t = {r["kernel"]: r for r in profsum.trace_table(str(tmp_path / "x_kernel_trace.csv"))}
    inner, outer = t["k_row_forward<float,11,0,0,5>"], t["k_row_forward<float,11,0,0,5>:outer"]
    assert inner["calls"] == 6 and inner["working_calls"] == 5 and abs(inner["working_avg_us"] - 16.0) < 1e-9
    assert outer["calls"] == 2 and abs(outer["working_avg_us"] - 40.0) < 1e-9
    # other kernels keep their long launches
    k2 = "void rdk::k_row_forward<double, 11, 0, 0, 1>(rdk::Slot* const*)"
    _write_trace(tmp_path / "y_kernel_trace.csv", [(k2, 0, 10000), (k2, 20000, 30000), (k2, 40000, 70000)])
    t2 = profsum.trace_table(str(tmp_path / "y_kernel_trace.csv"))
    assert len(t2) == 1 and t2[0]["working_calls"] == 3


def test_traffic_scaling_by_the_calibration_copy(tmp_path):
    k = "void rdk::k_upd<float, 11, 0, 0, 1>(rdk::Slot* const*)"
    cal = "void at::native::neg_kernel_cuda(at::TensorIteratorBase&)"
    for sub, counter, cal_kib, k_kib in (("f", "FETCH_SIZE", 512, 100), ("w", "WRITE_SIZE", 1024, 50)):
        d = tmp_path / sub
        d.mkdir()
        with open(d / "x_counter_collection.csv", "w") as f:
            f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            f.write('1,"%s",%s,%d\n' % (cal, counter, cal_kib))
            f.write('2,"%s",%s,%d\n' % (k, counter, k_kib))
    out = subprocess.run([sys.executable, "-m", "paper_2305_03945_amd.profsum", "traffic", str(tmp_path / "f"),
                          str(tmp_path / "w"), "x", str(1024 * 1024)], capture_output=True, text=True, cwd=ROOT,
                         check=True).stdout
    js = json.loads(out.strip().splitlines()[-1])
    # the copy moves 1 MiB each way: FETCH_SIZE read half of it (factor 2), WRITE_SIZE all (factor 1)
    assert abs(js["fetch_factor"] - 2.0) < 1e-12 and abs(js["write_factor"] - 1.0) < 1e-12
    assert abs(js["kernels"]["k_upd<float,11,0,0,1>"]["hbm_bytes"] - (100 * 1024 * 2 + 50 * 1024)) < 1e-6


def test_counters_average_working_dispatches_by_the_first_counter(tmp_path):
    k = "void rdk::k_row_forward<float, 11, 0, 0, 5>(rdk::Slot* const*)"
    rows = []
    # four inner launches (cycles 100, instructions 10), one outer update (cycles 300,
    # instructions 40) and one launch that found the slot finished (cycles 2)
    for i, (cyc, ins) in enumerate([(100, 10)] * 4 + [(300, 40), (2, 0)]):
        rows += [(i, "SQ_WAVE_CYCLES", cyc), (i, "SQ_INSTS_VALU", ins)]
    other = "rdk::k_copy_out(rdk::Slot* const*, double*, unsigned long)"
    with open(tmp_path / "x_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, c, v in rows:
            f.write('%d,"%s",%s,%d\n' % (i, k, c, v))
        f.write('9,"%s",SQ_WAVE_CYCLES,7\n' % other)
    t = profsum.counters_table(str(tmp_path / "x_counter_collection.csv"), ["SQ_WAVE_CYCLES", "SQ_INSTS_VALU"])
    assert t["rdk::k_copy_out"]["SQ_WAVE_CYCLES"] == 7
    inner, outer = t["k_row_forward<float,11,0,0,5>"], t["k_row_forward<float,11,0,0,5>:outer"]
    assert inner["dispatches"] == 5 and inner["working"] == 4
    assert inner["SQ_WAVE_CYCLES"] == 100 and inner["SQ_INSTS_VALU"] == 10
    assert outer["working"] == 1 and outer["SQ_INSTS_VALU"] == 40


def test_source_hash_ignores_comments(tmp_path):
    a, b = tmp_path / "a", tmp_path / "b"
    a.mkdir()
    b.mkdir()
    (a / "k.h").write_text("int f() { return 1; }  // one\n\n// note\n")
    (b / "k.h").write_text("// other note\nint f() { return 1; }\n")
    assert profsum.source_hash(str(a)) == profsum.source_hash(str(b))
    (b / "k.h").write_text("int f() { return 2; }\n")
    assert profsum.source_hash(str(a)) != profsum.source_hash(str(b))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
