"""Host logic of bench.py: the counter and kernel-trace summaries, read from
CSV files laid out as rocprofv3 writes them (nested under host and process
folders), with request counts chosen so that every byte figure is known."""
import csv
import os

import bench


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, sub, per_kernel):
    """per_kernel: {kernel name: {counter: value}} -> one dispatch each."""
    rows, trace = [], []
    for i, (name, cs) in enumerate(per_kernel.items()):
        for c, v in cs.items():
            rows.append([i, name, c, v])
        trace.append([name, 1000 * i, 1000 * i + 500])  # 0.5 us each
    _write(os.path.join(d, sub, "host", "123", "run_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    _write(os.path.join(d, sub, "host", "123", "run_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)


def test_pmc_summary_bytes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    copy = bench.COPY_MIB * 2 ** 20
    d = str(tmp_path / "prof")
    names = {"copy": "__amd_rocclr_copyBuffer", "gather": "void at::native::indexSelectLargeIndex",
             "field": "void k_field<1, 64, 32, 1>(StepArgs)"}
    # the copy: 128-byte reads and 64-byte writes; the kernel: reads of every
    # size and some 32-byte writes
    rd = {names["copy"]: {"TCC_EA0_RDREQ_sum": copy / 128, "TCC_EA0_RDREQ_32B_sum": 0,
                          "TCC_EA0_RDREQ_64B_sum": 0, "TCC_EA0_RDREQ_128B_sum": copy / 128},
          names["gather"]: {"TCC_EA0_RDREQ_sum": 1000, "TCC_EA0_RDREQ_32B_sum": 0,
                            "TCC_EA0_RDREQ_64B_sum": 1000, "TCC_EA0_RDREQ_128B_sum": 0},
          names["field"]: {"TCC_EA0_RDREQ_sum": 1000, "TCC_EA0_RDREQ_32B_sum": 100,
                           "TCC_EA0_RDREQ_64B_sum": 600, "TCC_EA0_RDREQ_128B_sum": 300}}
    wr = {names["copy"]: {"TCC_EA0_WRREQ_sum": copy / 64, "TCC_EA0_WRREQ_64B_sum": copy / 64},
          names["gather"]: {"TCC_EA0_WRREQ_sum": 0, "TCC_EA0_WRREQ_64B_sum": 0},
          names["field"]: {"TCC_EA0_WRREQ_sum": 30, "TCC_EA0_WRREQ_64B_sum": 10}}
    l2 = {n: {"TCC_HIT_sum": 3, "TCC_MISS_sum": 1} for n in names.values()}
    sq = {n: {"MfmaUtil": 12.5, "SQ_INSTS_VALU_MFMA_MOPS_BF16": 2} for n in names.values()}
    st = {n: {"SQ_WAVE_CYCLES": 100, "SQ_WAIT_ANY": 50, "SQ_ACTIVE_INST_VALU": 7,
              "SQ_ACTIVE_INST_LDS": 4} for n in names.values()}
    for sub, tab in (("rd", rd), ("wr", wr), ("l2", l2), ("sq", sq), ("st", st)):
        _counters(d, sub, tab)
    bench.pmc_summary(d, "unit", 5)
    lines = open(bench.traffic_file("unit")).read().splitlines()
    assert any("counted reads 1.0000, writes 1.0000 of its bytes; unsized read requests 0;" in l
               for l in lines)
    row = next(l.split() for l in lines if l.startswith("k_field "))
    read = 32 * 100 + 64 * 600 + 128 * 300
    write = 32 * 20 + 64 * 10
    assert (float(row[2]), float(row[3]), float(row[4])) == (read, write, read + write)
    assert float(row[7]) == 0.75 and float(row[8]) == 0.125 and float(row[9]) == 1024
    # the stall table repeats the kernel names after the byte table
    stall = [l.split() for l in lines if l.startswith("k_field ")][1]
    assert float(stall[2]) == 0.5 and float(stall[4]) == 0.07
    # a current summary feeds the benchmark's traffic figure; a stale one not
    assert bench.traffic_of("unit", ["k_field"]) == read + write
    with open(bench.traffic_file("unit"), "w") as fh:
        fh.write("\n".join(l if not l.startswith("kernel_source") else
                           "kernel_source_sha256_16 0000" for l in lines))
    assert bench.traffic_of("unit", ["k_field"]) is None


def test_trace_summary_table(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    d = str(tmp_path / "trace")
    _write(os.path.join(d, "host", "9", "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
            "StdDev"],
           [["k_pack(StepArgs, int)", 10, 80000, 8000, 10.0, 7000, 9000, 1],
            ["void k_field<1, 64, 32, 1>(StepArgs)", 10, 720000, 72000, 90.0, 70000, 75000, 1]])
    bench.trace_summary(d, "torus1", 100, 10)
    text = open(os.path.join(tmp_path, "profiles", "step_kernels_torus1.txt")).read()
    body = [l.split() for l in text.splitlines() if not l.startswith("#")
            and not l.startswith("kernel_source")]
    assert body[0][:2] == ["k_field<1,", "64,"] and body[0][-5:] == ["10", "72.00", "70.00",
                                                                     "75.00", "90.00"]
    assert body[1][0] == "k_pack(StepArgs," and body[1][-4] == "8.00"
    assert "--steps 100 --warmup 10 --only-headline --streams 1" in text


def _fake_psnr(monkeypatch, batched):
    """equal_psnr over synthetic curves: the plain path rises 0.1 dB over the
    steps from a per-seed base; `batched(step, base)` gives the batched path."""
    import types
    import paper_2304_05735_amd as pk
    monkeypatch.setattr(pk, "BATCH_ALL", "all", raising=False)
    monkeypatch.setattr(pk, "BATCH_PER_OBJECT", "per", raising=False)
    monkeypatch.setattr(pk, "PREC_FP32", 0, raising=False)

    def make_ctx(wl, pr, mode, graph, seed=0, **k):
        return types.SimpleNamespace(key=(pr, mode, seed)), None, None

    def curve(q, wl, ids, rays, n, chunk):
        pr, mode, seed = q.key
        base = 27.0 + 0.4 * seed
        f = (lambda s: batched(s, base)) if (mode == "all" and pr == 1) else \
            (lambda s: base + 0.1 * s / 2000)
        return [(s, f(s)) for s in range(chunk, n + 1, chunk)]

    monkeypatch.setattr(bench, "make_ctx", make_ctx)
    monkeypatch.setattr(bench, "psnr_curve", curve)
    wl = types.SimpleNamespace(eval_views=[0])
    return bench.equal_psnr(wl, [0], [1], 1, 2000, 250, 2.0, 6.0, seeds=(0, 1))


def test_equal_psnr_rule(monkeypatch):
    # within 0.1 dB after the steps: the ratio of rates at equal steps
    out = _fake_psnr(monkeypatch, lambda s, b: b + 0.1 * s / 2000 - 0.05)
    assert out["speedup_at_equal_psnr"] == 3.0 and out["delta_psnr"] == -0.05
    assert len(out["curve_batched"]) == 16 and len(out["curve_plain_fp32"]) == 8
    # below: the batched path trains on and its time to the plain path's PSNR
    # (27.3 dB; its mean is 26.8 + 0.15 dB per 1000 steps, first at or above
    # it at the 3500-step checkpoint) is compared with the plain path's 2000
    out = _fake_psnr(monkeypatch, lambda s, b: b - 0.4 + 0.3 * s / 2000)
    assert out["psnr_batched"] == 27.1 and out["steps_batched_to_target"] == 3500
    assert out["speedup_at_equal_psnr"] == round(2000 * 6.0 / (3500 * 2.0), 3)
    # above: reached before the steps end
    out = _fake_psnr(monkeypatch, lambda s, b: b + 0.3 * s / 1000)
    assert out["steps_batched_to_target"] == 500
    # never reached within twice the steps: null
    out = _fake_psnr(monkeypatch, lambda s, b: b - 1.0)
    assert out["steps_batched_to_target"] is None and out["speedup_at_equal_psnr"] is None
