"""The profile and counter summaries bench.py writes from rocprofv3 output
(no GPU): kernel times per grid from the trace, HBM bytes scaled by what the
counters read for the 256 MiB copy, medians per kernel and the MFMA-busy
fraction.  Inputs are small CSV files in rocprofv3's column layout."""
import argparse
import csv
import json
import os

import bench

NEAR = "void fmm::k_near_pair<float, 1>(int const*, int)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _args(**kw):
    base = dict(summary_title="t", summary_cmd=["cmd"], summary_note=[], traffic_out="", summary_out="")
    base.update(kw)
    return argparse.Namespace(**base)


def test_profile_summary_splits_the_near_launches_by_grid_and_scales_counter_bytes(tmp_path):
    tr, fe, wr = (str(tmp_path / d) for d in ("trace", "fetch", "write"))
    _write(f"{tr}/run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [[NEAR, 4, 4000, 1000], [COPY, 1, 50, 50]])
    # two launches of 100 workgroups (1000, 2000 ns) and two of 10 (500, 700 ns)
    trace = [[NEAR, t0, t0 + d, 64, 64 * g] for t0, d, g in ((0, 1000, 100), (5000, 2000, 100),
                                                            (9000, 500, 10), (12000, 700, 10))]
    _write(f"{tr}/run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X",
                                          "Grid_Size_X"], trace)
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"]
    # the copy reads 128 MiB and writes 256 MiB as counted: scales 2 and 1
    _write(f"{fe}/run_counter_collection.csv", hdr,
           [[1, COPY, 1 << 20, 256, "FETCH_SIZE", 131072.0]] +
           [[2 + i, NEAR, 64 * g, 64, "FETCH_SIZE", v] for i, (g, v) in enumerate(((100, 10.0), (100, 30.0),
                                                                                     (10, 4.0), (10, 4.0)))])
    _write(f"{wr}/run_counter_collection.csv", hdr,
           [[1, COPY, 1 << 20, 256, "WRITE_SIZE", 262144.0]] +
           [[2 + i, NEAR, 64 * g, 64, "WRITE_SIZE", v] for i, (g, v) in enumerate(((100, 5.0), (100, 5.0),
                                                                                     (10, 1.0), (10, 3.0)))])
    out_md, out_json = str(tmp_path / "p.md"), str(tmp_path / "traffic.json")
    bench.summarize_profile(_args(summarize_profile=[tr, fe, wr], summary_out=out_md, traffic_out=out_json))
    md = open(out_md).read()
    assert "| `void fmm::k_near_pair<float, 1>` | 100 | 2 | 1.50 | 1.00 | 2.00 |" in md
    assert "| `void fmm::k_near_pair<float, 1>` | 10 | 2 | 0.60 | 0.50 | 0.70 |" in md
    rec = json.load(open(out_json))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    t = rec["traffic"]
    # medians over the dispatches of each grid, in KiB, times the scales
    assert t["void fmm::k_near_pair<float, 1> @100"]["read_bytes"] == 20.0 * 1024 * 2
    assert t["void fmm::k_near_pair<float, 1> @100"]["write_bytes"] == 5.0 * 1024
    assert t["void fmm::k_near_pair<float, 1> @10"]["read_bytes"] == 4.0 * 1024 * 2
    assert t["void fmm::k_near_pair<float, 1> @10"]["write_bytes"] == 2.0 * 1024
    assert t["void fmm::k_near_pair<float, 1>"]["read_bytes"] == 7.0 * 1024 * 2
    assert len(rec["kernels_code_sha256"]) == 64


def test_counter_summary_gives_medians_and_the_mfma_busy_fraction(tmp_path):
    p1 = str(tmp_path / "p1")
    gemm = "void fmm::k_gemm_bf3<3, 64>(fmm::GemmArgs)"
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"]
    rows = []
    for i, (gui, busy) in enumerate(((80000, 1024000), (80000, 2048000), (160000, 3072000))):
        rows += [[i, gemm, 256 * 100, 256, "GRBM_GUI_ACTIVE", gui], [i, gemm, 256 * 100, 256,
                                                                     "SQ_VALU_MFMA_BUSY_CYCLES", busy]]
    _write(f"{p1}/run_counter_collection.csv", hdr, rows)
    out = str(tmp_path / "c.md")
    bench.summarize_counters(_args(summarize_counters=[p1], summary_out=out, summary_note=["a note"]))
    md = open(out).read()
    # medians: GRBM 80,000, busy 2,048,000 -> 2,048,000 / (80,000 / 8 x 1,024) = 0.2
    assert "| `void fmm::k_gemm_bf3<3, 64>` | 3 | 80,000 | 2,048,000 | 0.200 |" in md
    assert md.rstrip().endswith("a note")


def test_kernel_digest_ignores_comments_and_whitespace_only(tmp_path):
    a, b, c = (str(tmp_path / f) for f in ("a.hip", "b.hip", "c.hip"))
    open(a, "w").write("// head\n__global__ void k(float *x) {\n  x[0] = 1.f;  /* set */\n}\n")
    open(b, "w").write("/* another\n   head */\n__global__ void k(float *x)\n{ x[0] = 1.f; // set\n}\n")
    open(c, "w").write("__global__ void k(float *x) {\n  x[0] = 2.f;\n}\n")
    assert bench.kernel_source_digest(a) == bench.kernel_source_digest(b)
    assert bench.kernel_source_digest(a) != bench.kernel_source_digest(c)
