"""Host-side parts of bench.py: the one-GPU guard and the lookup of the HBM
byte counts, which are reported only for the kernel sources they were
measured on (no GPU calls)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout.strip() == ""


def test_source_hash_covers_every_kernel_source(tmp_path):
    b = _bench_module()
    h = b.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert b.kernel_source_hash() == h   # deterministic
    # a copy of the sources: a comment or spacing edit keeps the hash, a code
    # edit changes it
    csrc = os.path.join(ROOT, "paper_2605_30342_amd", "csrc")
    dst = tmp_path / "paper_2605_30342_amd" / "csrc"
    dst.mkdir(parents=True)
    names = sorted(os.listdir(csrc))
    for n in names:
        (dst / n).write_bytes(open(os.path.join(csrc, n), "rb").read())
    b.ROOT = str(tmp_path)
    assert b.kernel_source_hash() == h
    last = dst / names[-1]
    orig = last.read_bytes()
    last.write_bytes(orig + b"\n// a comment\n/* another */  \n")
    assert b.kernel_source_hash() == h
    last.write_bytes(orig + b"\nstatic int extra_symbol;\n")
    assert b.kernel_source_hash() != h


def test_strip_comments_keeps_literals():
    b = _bench_module()
    src = 'int a = 1; // c\n/* x */ const char *s = "a//b /*c*/"; char q = \'"\'; int b; /* y\n z */ x'
    assert b.strip_comments(src) == 'int a = 1; const char *s = "a//b /*c*/"; char q = \'"\'; int b; x'


def test_traffic_is_reported_only_for_matching_sources(tmp_path):
    b = _bench_module()
    (tmp_path / "profiles").mkdir()
    doc = {"source_hash": "0123456789abcdef",
           "workloads": {"room": {"build": {"raster_vis": {"read": 100000, "write": 23456, "launches": 1}},
                                  "query": {"project": {"read": 10, "write": 20, "launches": 1}}}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(doc))
    b.ROOT = str(tmp_path)
    b.kernel_source_hash = lambda: "0123456789abcdef"
    assert b.traffic_for("raster_vis") == 123456
    assert b.traffic_for("raster_uq") is None           # no entry
    assert b.stage_traffic("room", "query")["project"]["write"] == 20
    assert b.stage_traffic("precision", "query") is None
    b.kernel_source_hash = lambda: "fedcba9876543210"
    assert b.traffic_for("raster_vis") is None          # measured on other sources
    assert b.stage_traffic("room", "query") is None
    (tmp_path / "profiles" / "traffic.json").write_text("not json")
    assert b.traffic_for("raster_vis") is None


def test_stage_labels_follow_the_launch_order():
    """Kernels of one query call, in launch order, map to the library's
    stages; the radix passes before the emission are the depth sort, those
    after it the tile sort."""
    b = _bench_module()
    seq = ["__amd_rocclr_copyBuffer", "k_fill_u32(unsigned*)", "void k_count<float>(GaussIn<float>)",
           "k_scan_reduce(x)", "k_scan_blocks(x)", "k_scan_down(x)", "void k_project<float, float, 1, 3, false>(x)",
           "k_radix_hist(x)", "k_radix_scan(x)", "k_radix_scatter(x)", "k_radix_hist(x)", "k_radix_scan(x)",
           "k_radix_scatter(x)", "k_scan_reduce(x)", "k_scan_blocks(x)", "k_scan_down(x)", "k_fill_u32(unsigned*)",
           "k_emit(x)", "k_radix_hist(x)", "k_radix_scan(x)", "k_radix_scatter(x)", "k_ranges(x)",
           "void k_raster_uq<256, false, false, false, false>(x)", "k_scores(x)", "k_argmax(x)"]
    lab = b.label_stages(seq)
    assert lab[0] == "other" and lab[1:6] == ["cull"] * 5 and lab[6] == "project"
    assert lab[7:13] == ["sort_depth"] * 6 and lab[13:18] == ["emit"] * 5
    assert lab[18:21] == ["sort_tile"] * 3 and lab[21] == "ranges" and lab[22] == "raster_uq"
    assert lab[23:] == ["scores", "scores"]


def test_hbm_fractions_sum_the_binning_stages():
    b = _bench_module()
    tr = {"project": {"read": 4e9, "write": 4e9}, "sort_depth": {"read": 8e9, "write": 0},
          "raster_uq": {"read": 1e9, "write": 0}}
    r = b.hbm_fractions(tr, {"project": 2.0, "sort_depth": 2.0, "raster_uq": 1.0})
    assert abs(r["project"]["frac"] - 0.5) < 1e-9           # 8 GB in 2 ms = 4 TB/s
    assert abs(r["projection_and_binning"]["frac"] - 0.5) < 1e-9
    assert r["projection_and_binning"]["bytes"] == 16e9


def test_last_calls_pick_one_build_and_the_timed_query():
    """The counter summary takes the last one-pass build and the last query
    that does not count pairs, each from its view-table upload to its last
    kernel (trailing copies of other work left out)."""
    b = _bench_module()
    call = ["__amd_rocclr_copyBuffer", "k_fill_u32(x)", "void k_count<float>(x)", "k_project(x)"]
    rows = []
    seqs = [call + ["void k_raster_vis<64>(x)", "k_vf_accum(x)"],
            call + ["void k_raster_uq<256, false, false, false, false>(x)", "k_scores(x)", "k_argmax(x)"],
            call + ["void k_raster_uq<256, false, true, false, false>(x)", "k_scores(x)"],
            ["__amd_rocclr_copyBuffer", "void at::vectorized_elementwise_kernel<4>(x)"]]
    for seq in seqs:
        rows += [(len(rows) + i, n, 0.0, 0, 1) for i, n in enumerate(seq)]
    bld, qry = b._last_calls(rows)
    assert [b._kernel_base(r[1]) for r in bld][-2:] == ["k_raster_vis", "k_vf_accum"] and len(bld) == 6
    assert "false, false, false, false" in qry[4][1] and b._kernel_base(qry[-1][1]) == "k_argmax"
