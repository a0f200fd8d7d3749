"""Host logic of the profile summaries: HBM bytes per launch from counter
runs (the copy-scaled FETCH_SIZE / WRITE_SIZE figures and the exact count by
read-request size)."""

import csv
import json

import pytest

from paper_2309_11273_amd import profsum

COPY = "void at::native::vectorized_elementwise_kernel<4, MulFunctor<float> >(int, float*)"
P1 = "void pdk::k_tpass1_f32<3, true, 1>(pdk::StepArgs, int, pdk::KEnt const*, pdk::KEnt1 const*)"
P2 = "void pdk::k_tpass2_f32<3, true, 1>(pdk::StepArgs, int, pdk::KEnt1 const*)"


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def _req_rows(kernel, n32, n64, n128):
    return [(kernel, "TCC_EA0_RDREQ_32B_sum", n32), (kernel, "TCC_EA0_RDREQ_64B_sum", n64),
            (kernel, "TCC_EA0_RDREQ_128B_sum", n128), (kernel, "TCC_EA0_RDREQ_sum", n32 + n64 + n128)]


def test_copy_scaled_traffic(tmp_path):
    # the copy reads 1 MiB and FETCH_SIZE shows half of it; WRITE_SIZE all of it
    cb = 1 << 20
    _csv(tmp_path / "f.csv", [(COPY, "FETCH_SIZE", 512), (P1, "FETCH_SIZE", 100), (P1, "FETCH_SIZE", 300)])
    _csv(tmp_path / "w.csv", [(COPY, "WRITE_SIZE", 1024), (P1, "WRITE_SIZE", 50)])
    out = tmp_path / "t.json"
    db = profsum.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), cb, "wl", str(out))
    e = db["k_tpass1_f32@wl"]
    assert e["fetch_bytes"] == 200 * 1024 * 2 and e["write_bytes"] == 50 * 1024
    assert e["bytes_per_launch"] == 200 * 1024 * 2 + 50 * 1024
    assert e["source_sha"] == profsum.kernel_source_hash("k_tpass1_f32")
    assert json.load(open(out)) == db


def test_exact_bytes_by_request_size(tmp_path):
    cb = 1 << 20
    out = tmp_path / "t.json"
    sha = profsum.kernel_source_hash("k_tpass1_f32")
    json.dump({"k_tpass1_f32@wl": {"bytes_per_launch": 1, "write_bytes": 1000, "source_sha": sha},
               "k_tpass2_f32@wl": {"bytes_per_launch": 1, "write_bytes": 7, "source_sha": "stale"}},
              open(out, "w"))
    # two dispatches of pass 1 (mean taken), one of pass 2, the copy all 128-byte requests
    _csv(tmp_path / "r.csv", _req_rows(COPY, 0, 0, cb // 128) + _req_rows(P1, 3, 10, 20) + _req_rows(P1, 5, 30, 40)
         + _req_rows(P2, 0, 1, 1))
    db = profsum.requests(str(tmp_path / "r.csv"), cb, "wl", str(out))
    rd = 32 * 4 + 64 * 20 + 128 * 30
    assert db["k_tpass1_f32@wl"]["read_bytes_exact"] == rd
    assert db["k_tpass1_f32@wl"]["bytes_per_launch_exact"] == rd + 1000
    # an entry taken on other kernel sources is left as it is
    assert "read_bytes_exact" not in db["k_tpass2_f32@wl"]


def test_request_counts_must_reproduce_the_copy(tmp_path):
    cb = 1 << 20
    _csv(tmp_path / "r.csv", _req_rows(COPY, 0, cb // 128, 0) + _req_rows(P1, 1, 1, 1))
    with pytest.raises(SystemExit):
        profsum.requests(str(tmp_path / "r.csv"), cb, "wl", str(tmp_path / "t.json"))


def test_tail_averages_the_last_dispatches(tmp_path):
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        # out of time order on purpose: the last dispatches are the latest starts
        for start, dur in ((300, 5000), (100, 1000), (200, 3000), (400, 7000)):
            w.writerow({"Kernel_Name": P1, "Start_Timestamp": start, "End_Timestamp": start + dur})
        w.writerow({"Kernel_Name": COPY, "Start_Timestamp": 0, "End_Timestamp": 99999})
    md = profsum.tail_md(str(path), 2)
    assert "| `k_tpass1_f32<3, true, 1>` | 4 | 2 | 6.00 |" in md
    assert "MulFunctor" not in md
