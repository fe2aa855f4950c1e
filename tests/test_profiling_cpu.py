"""The rocprofv3 summaries behind the bench line's traffic, L2 and record checks, on small
synthetic counter files with known answers (CPU only)."""

import csv

import pytest

from paper_2307_03017_amd import profiling as P

COLS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value", "Start_Timestamp",
        "End_Timestamp"]
GRAD = "void hsgd::(anonymous namespace)::k_grad_shift<0, 32, true>(void const*, int, int)"
COPY = "void hsgd::(anonymous namespace)::k_convert<0, 0>(void const*, void*, long)"


def write_csv(path, rows, cols=COLS):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: r.get(c, 0) for c in cols})
    return str(path)


def counter(d, name, grid, ctr, value, t0=0, t1=0):
    return dict(Dispatch_Id=d, Kernel_Name=name, Grid_Size=grid, Counter_Name=ctr, Counter_Value=value,
                Start_Timestamp=t0, End_Timestamp=t1)


def test_short_name():
    assert P.short_name(GRAD) == "k_grad_shift<0, 32, true>"
    assert P.short_name("k_downsample") == "k_downsample"
    torch_fill = ("void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>, "
                  "std::array<char*, 1ul> >(int, at::native::FillFunctor<float>, std::array<char*, 1ul>)")
    assert P.short_name(torch_fill) == ("at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>, "
                                        "std::array<char*, 1ul> >")


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    # a 256 MiB copy (copy_bytes counts both directions: 512 MiB) whose FETCH_SIZE reads half
    # of its bytes and whose WRITE_SIZE reads all of them: factors 2 and 1
    half = 256 * 1024  # KiB
    fetch = [counter(1, COPY, 100, "FETCH_SIZE", half // 2),
             counter(2, GRAD, 1000, "FETCH_SIZE", 10.0), counter(3, GRAD, 1000, "FETCH_SIZE", 30.0),
             counter(4, GRAD, 4000, "FETCH_SIZE", 100.0)]
    write = [counter(1, COPY, 100, "WRITE_SIZE", half),
             counter(2, GRAD, 1000, "WRITE_SIZE", 5.0), counter(3, GRAD, 1000, "WRITE_SIZE", 7.0),
             counter(4, GRAD, 4000, "WRITE_SIZE", 50.0)]
    t = P.traffic(write_csv(tmp_path / "f.csv", fetch), write_csv(tmp_path / "w.csv", write), "k_grad_shift",
                  2 * 256 * 1024 * 1024)
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    by_grid = {l["grid"]: l for l in t["launches"]}
    assert by_grid[1000]["read_bytes"] == pytest.approx(20.0 * 1024 * 2.0)     # mean of 10 and 30 KiB, x2
    assert by_grid[1000]["write_bytes"] == pytest.approx(6.0 * 1024)
    assert by_grid[4000]["read_bytes"] == pytest.approx(100.0 * 1024 * 2.0)
    mean = (20 * 2 + 6 + 100 * 2 + 50) * 1024 / 2
    assert t["hbm_bytes_per_launch"] == pytest.approx(mean)
    assert "FETCH_SIZE x 2.000" in P.traffic_md(t, "cmd")


def test_traffic_without_the_copy_kernel_is_refused(tmp_path):
    rows = [counter(2, GRAD, 1000, "FETCH_SIZE", 10.0)]
    f = write_csv(tmp_path / "f.csv", rows)
    with pytest.raises(SystemExit):
        P.traffic(f, f, "k_grad_shift", 1 << 20)


def test_l2_pools_template_instances_and_keeps_grids_apart(tmp_path):
    other = GRAD.replace("<0, 32, true>", "<1, 32, true>")
    rows = [counter(1, GRAD, 1000, "TCC_HIT_sum", 30), counter(1, GRAD, 1000, "TCC_MISS_sum", 10),
            counter(2, GRAD, 1000, "TCC_HIT_sum", 50), counter(2, GRAD, 1000, "TCC_MISS_sum", 10),
            counter(3, other, 2000, "TCC_HIT_sum", 0), counter(3, other, 2000, "TCC_MISS_sum", 100)]
    t = P.l2(write_csv(tmp_path / "l2.csv", rows))
    by = {(r["kernel"], r["grid"]): r for r in t["rows"]}
    assert by[("k_grad_shift<0, 32, true>", 1000)]["dispatches"] == 2
    assert by[("k_grad_shift<0, 32, true>", 1000)]["hit_rate"] == pytest.approx(80 / 100)
    assert by[("k_grad_shift<1, 32, true>", 2000)]["hit_rate"] == 0.0
    assert t["hit_rate"]["k_grad_shift"] == pytest.approx(80 / 200)


def test_sq_slot_load_and_clock(tmp_path):
    # 8 XCDs of busy cycles summing to 8 x 1000: a 1000-cycle launch over 1 us (1 GHz); 4 SIMDs
    # issuing 1000 VALU instructions of 4 cycles each are fully loaded
    vals = dict(SQ_INSTS_VALU=1000, SQ_INSTS_SALU=500, SQ_INSTS_LDS=40, SQ_WAVES=8, SQ_WAVE_CYCLES=4000,
                SQ_ACTIVE_INST_VALU=1000, SQ_WAIT_INST_ANY=1000, SQ_BUSY_CYCLES=1000, GRBM_GUI_ACTIVE=8000)
    rows = [counter(7, GRAD, 512, c, v, 1_000_000, 1_001_000) for c, v in vals.items()]
    rows.append(counter(8, COPY, 512, "SQ_WAVES", 1, 0, 1))               # another kernel: ignored
    agent = write_csv(tmp_path / "agent.csv", [dict(Simd_Count=0, Num_Xcc=0), dict(Simd_Count=4, Num_Xcc=8)],
                      cols=["Simd_Count", "Num_Xcc"])
    t = P.sq(write_csv(tmp_path / "sq.csv", rows), agent, "k_grad_shift")
    (r,) = t["rows"]
    assert (t["simds"], t["xcds"]) == (4, 8)
    assert r["us"] == pytest.approx(1.0) and r["clock_ghz"] == pytest.approx(1.0)
    assert r["valu_per_wave"] == pytest.approx(125) and r["salu_per_wave"] == pytest.approx(62.5)
    assert r["valu_slot_load"] == pytest.approx(1.0) and r["salu_slot_load"] == pytest.approx(0.5)
    assert r["wait_share"] == pytest.approx(0.25)
    assert "| 100.0% | 50.0% | 25.0% |" in P.sq_md(t, "cmd")


def test_source_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    src = tmp_path / "csrc"
    src.mkdir()
    files = {f: "int f(int x) { return x + 1; }\n" for f in P.DEFAULT_SOURCES}
    for f, text in files.items():
        (src / f).write_text(text)
    monkeypatch.setattr(P, "_PKG", str(tmp_path))
    h0 = P.kernel_source_hash("k_grad_shift")
    f0 = P.DEFAULT_SOURCES[0]
    (src / f0).write_text("// a note\nint f(int x) {  /* block\n comment */ return x + 1;\n}\n")
    assert P.kernel_source_hash("k_grad_shift") == h0
    (src / f0).write_text("int f(int x) { return x + 2; }\n")
    assert P.kernel_source_hash("k_grad_shift") != h0
