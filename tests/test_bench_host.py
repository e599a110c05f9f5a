"""Host-side logic of bench.py: the kernel table and the roofline object
(no GPU): per-launch timings of each preconditioner form map to the right
kernels, work figures and peaks."""
import bench


def test_fast_form_roofline_picks_dominant_hbm_kernel():
    N = M = 8192
    launches = [("prologue", 0.004), ("rows_dct2", 0.13), ("transpose", 0.09), ("cols", 0.26),
                ("transpose", 0.09), ("rows_dct3", 0.19), ("partials", 0.014)]
    kern = bench.kernel_table(None, launches, 0.22, "bf16", N, M)
    assert kern["transpose_kernel"]["launches"] == 2
    assert abs(kern["transpose_kernel"]["ms"] - 0.18) < 1e-12
    assert kern["fct_cols_kernel"]["bytes_per_launch"] == 8 * N * M
    assert kern["stencil_kernel"]["bytes_per_launch"] == 16 * N * M
    roof = bench.roofline(kern, "bf16")
    assert roof["kernel"] == "fct_cols_kernel" and roof["bound"] == "hbm"
    assert abs(roof["achieved"] - 8 * N * M / 0.26e-3 / 1e9) < 0.1
    assert roof["peak"] == 8000.0 and abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-4


def test_folded_form_roofline_reports_dense_equivalent_and_executed():
    N = M = 8192
    launches = [("prologue", 0.004), ("butterfly", 0.05)] + [("product", 0.4)] * 8 + [("dots", 0.1)]
    kern = bench.kernel_table(None, launches, 0.22, "bf16", N, M)
    roof = bench.roofline(kern, "bf16")
    assert roof["kernel"] == "gemm_nt_kernel" and roof["bound"] == "mfma"
    dense = 4.0 * N * M * (N + M) / 8
    assert roof["flops_per_launch"] == dense
    assert abs(roof["achieved"] - dense / 0.4e-3 / 1e12) < 0.01
    assert abs(roof["executed_TFLOPs"] - roof["achieved"] / 2) < 0.01


def test_f64_stencil_bytes_double():
    kern = bench.kernel_table(None, [("product", 1.0)] * 4, 0.5, "f64", 256, 256)
    assert kern["stencil_kernel"]["bytes_per_launch"] == 32 * 256 * 256
