"""Host-side logic of bench.py that needs no GPU: the source hash the HBM
counter record is keyed by, and the record lookup."""
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
    h = rec["src_hash"]
    for cls, k in rec["kernels"].items():
        got = bench._traffic(cls, h)
        assert got == k["bytes_per_launch"] and got > 0
    # a record taken on other kernel sources is not reported
    assert bench._traffic("col_fft", "0" * 16) is None
    assert bench._traffic("no_such_class", h) is None


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
