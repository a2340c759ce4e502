"""The rocprofv3 summariser's cold/warm split (host logic, no GPU)."""
from paper_1511_02494_amd.profiling import FLUSH, cold_flags, cold_warm_means

F = FLUSH + "(unsigned int __vector(4)*, long)"
A = "void spmvsel::k_rowstream_slices<double, 1, false>(...)"
B = "void spmvsel::k_slice_finish<double>(...)"
T = "void at::native::vectorized_elementwise_kernel<...>"


def test_cold_flags_follow_flushes():
    seq = [A, B, A, B, F, A, B, A, B, F, A, T, F, T, A, A, F, F, A]
    assert cold_flags(seq) == [False, False, False, False, False, True, True, False, False,
                               False, True, True, False, True, True, False, False, False, True]


def test_cold_warm_means():
    seq = [(A, 10.0), (B, 1.0), (F, 99.0), (A, 20.0), (B, 3.0), (A, 12.0), (B, None)]
    m = cold_warm_means(seq)
    assert m[A]["cold_n"] == 1 and m[A]["cold_mean"] == 20.0   # the second A starts a new execute
    assert m[A]["warm_n"] == 2 and m[A]["warm_mean"] == 11.0
    assert m[B]["cold_n"] == 1 and m[B]["cold_mean"] == 3.0 and m[B]["warm_mean"] == 1.0


def test_derived_shares_and_grid_grouping(tmp_path):
    """Counter means per (kernel, grid size), summed per dispatch over the
    rows rocprofv3 writes for it, and the derived shares of the busy time."""
    from paper_1511_02494_amd.profiling import counters_main, derived_columns
    m = {"GRBM_GUI_ACTIVE": 8 * 2400.0, "TA_TA_BUSY_sum": 256 * 1200.0,
         "TCC_HIT_sum": 3.0, "TCC_MISS_sum": 1.0,
         "TCP_TCC_READ_REQ_sum": 10.0, "TCP_TCC_READ_REQ_LATENCY_sum": 5000.0,
         "TCP_TOTAL_CACHE_ACCESSES_sum": 40.0}
    d = derived_columns(m)
    assert d["busy us (2.4 GHz)"] == 1.0
    assert d["address unit busy"] == 0.5
    assert d["L2 hit rate"] == 0.75
    assert d["L2 read latency (cycles)"] == 500.0 and d["L1 accesses per L2 read"] == 4.0
    run = tmp_path / "run"
    run.mkdir()
    rows = ["Dispatch_Id,Kernel_Name,Grid_Size,Counter_Name,Counter_Value"]
    for disp, grid, v in ((1, 64, 1.0), (2, 64, 3.0), (3, 128, 10.0)):
        rows += [f'{disp},"{A}",{grid},TA_TA_BUSY_sum,{v}', f'{disp},"{A}",{grid},TA_TA_BUSY_sum,{v}']
    rows.append(f'4,"{T}",64,TA_TA_BUSY_sum,7.0')
    (run / "x_counter_collection.csv").write_text("\n".join(rows) + "\n")
    out = tmp_path / "c.md"
    counters_main(["--dirs", str(run), "--cmds", "cmd", "--kernels", "void spmvsel::",
                   "--title", "t", "--by-grid", "--out", str(out)])
    text = out.read_text()
    assert "| 64 | 4 |" in text and "| 128 | 20 |" in text   # two rows per dispatch summed, then averaged
    assert "vectorized_elementwise" not in text
