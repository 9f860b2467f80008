"""Host-side logic of bench.py that needs no GPU: the source hash the HBM
counter record is keyed by, the record lookup, the counter-file reduction,
the search for the first iteration within the error bar, and the refusal of
a multi-GPU run."""
import csv
import json
import os

import bench


def test_src_hash_is_stable_and_short():
    a, b = bench._src_hash(), bench._src_hash()
    assert a == b and len(a) == 16
    int(a, 16)


def test_traffic_record_lookup():
    path = os.path.join(bench.ROOT, "profiles", "traffic.json")
    with open(path) as f:
        rec = json.load(f)
    for wl, w in rec["workloads"].items():
        h = w["src_hash"]
        for cls, k in w["classes"].items():
            got = bench._traffic(wl, cls, h)
            assert got == k["bytes_per_launch"] and got > 0
        # a record taken on other kernel sources is not reported
        assert bench._traffic(wl, "col_fft", "0" * 16) is None
        assert bench._traffic(wl, "no_such_class", h) is None
    assert bench._traffic("no_such_workload", "passb", "0" * 16) is None


def _pmc_csv(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w",
              newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name",
                    "Counter_Value"])
        for i, (k, v) in enumerate(rows):
            w.writerow([i, k, counter, v])


def test_traffic_from_counter_files(tmp_path):
    """FETCH_SIZE reads half the bytes of the calibration copy, WRITE_SIZE
    all of them: the factors 2 and 1 are found and applied per dispatch,
    and kernels are grouped into the bench's classes."""
    mib = 512
    kib = mib * 1024.0
    cf, cw = str(tmp_path / "cf"), str(tmp_path / "cw")
    _pmc_csv(cf, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", kib / 2)] * 3)
    _pmc_csv(cw, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", kib)] * 3)
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    _pmc_csv(f, "FETCH_SIZE", [("expdiag::passb_kernel<64, 0>", 1000.0),
                               ("expdiag::passb_kernel<64, 0>", 3000.0),
                               ("expdiag::col_kernel_host<256, 1>", 500.0)])
    _pmc_csv(w, "WRITE_SIZE", [("expdiag::passb_kernel<64, 0>", 100.0),
                               ("expdiag::passb_kernel<64, 0>", 300.0),
                               ("expdiag::col_kernel_host<256, 1>", 50.0)])
    out = str(tmp_path / "traffic.json")
    bench.traffic(f, w, cf, cw, "wl", mib=mib, path=out)
    with open(out) as fh:
        rec = json.load(fh)["workloads"]["wl"]
    assert abs(rec["fetch_factor"] - 2.0) < 1e-12
    assert abs(rec["write_factor"] - 1.0) < 1e-12
    pb = rec["classes"]["passb"]["bytes_per_launch"]
    assert abs(pb - (2.0 * 2000.0 + 200.0) * 1024.0) < 1e-6
    col = rec["classes"]["col_fft"]["bytes_per_launch"]
    assert abs(col - (2.0 * 500.0 + 50.0) * 1024.0) < 1e-6


def test_first_within_search():
    """Error curves that fall by 10x per iteration: the search finds each
    instance's first count within 1e-10, from a start above it (moves
    down), below it (moves up) and exactly at it."""
    first = [7, 12, 3]          # err(k) = 10^(first - 10 - k)
    state = {"caps": None}

    def run(caps):
        state["caps"] = list(caps)

    def errs():
        return [10.0 ** (f - 10 - k) for f, k in zip(first, state["caps"])]

    got = bench._first_within(run, errs, [10, 9, 3])
    assert got == first


def test_multi_gpu_request_is_refused(capsys):
    import sys
    argv = sys.argv
    sys.argv = ["bench.py", "--gpus", "2"]
    try:
        try:
            bench.main()
            raised = None
        except SystemExit as e:
            raised = e.code
    finally:
        sys.argv = argv
    assert raised == 2
    assert "one GPU" in capsys.readouterr().err
