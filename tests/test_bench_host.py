"""Host-side logic of bench.py: the kernel table and the roofline object
(no GPU): per-launch timings of one recorded PCG iteration map to the right
kernels, work figures and peaks."""
import bench


def test_fast_form_table_and_dominant_kernel():
    N = M = 8192
    px = N * M
    launches = [("stencil", 0.35), ("axpy", 0.36), ("prologue", 0.004), ("rows_dct2", 0.12),
                ("transpose", 0.1), ("cols", 0.2), ("transpose", 0.1), ("rows_dct3", 0.18),
                ("partials", 0.015)]
    kern = bench.kernel_table(launches, "f16", "fast", N, M, flexible=True)
    assert kern["transpose_kernel"]["launches"] == 2
    assert abs(kern["transpose_kernel"]["ms"] - 0.2) < 1e-12
    assert kern["transpose_kernel"]["bytes_per_launch"] == 4 * px      # FP16 storage
    assert kern["fct_rows_fwd_kernel"]["bytes_per_launch"] == 6 * px   # r FP32 in, T1 FP16 out
    assert kern["fct_rows_inv_kernel"]["bytes_per_launch"] == 14 * px  # T, r, q in; z out
    assert kern["stencil_kernel"]["bytes_per_launch"] == 24 * px
    assert kern["fct_cols_kernel"]["bound"] == "alu"
    roof = bench.roofline(kern, "f16")
    assert roof["kernel"] == "axpy_kernel" and roof["bound"] == "hbm"
    assert abs(roof["achieved"] - 24 * px / 0.36e-3 / 1e9) < 0.1
    assert roof["peak"] == 8000.0


def test_folded_form_rated_on_executed_flops():
    """The folded form executes 2NM(N+M) per application (half the dense
    4NM(N+M)); achieved and frac follow the executed flops, the dense
    equivalent is a side field."""
    N = M = 8192
    launches = ([("stencil", 0.35), ("axpy", 0.36), ("prologue", 0.004), ("butterfly", 0.05)]
                + [("product", 0.4)] * 8 + [("dots", 0.1)])
    kern = bench.kernel_table(launches, "bf16", "folded", N, M, flexible=True)
    roof = bench.roofline(kern, "bf16")
    assert roof["kernel"] == "gemm_nt_kernel" and roof["bound"] == "mfma"
    executed = 2.0 * N * M * (N + M) / 8
    assert roof["flops_per_launch"] == executed
    assert abs(roof["achieved"] - executed / 0.4e-3 / 1e12) < 0.01
    assert abs(roof["frac"] - roof["achieved"] / 2500.0) < 1e-4
    assert abs(roof["dense_equivalent_TFLOPs"] - 2 * roof["achieved"]) < 0.02


def test_fused_head_moves_the_iterate_update_to_the_last_pass():
    """With the CG update fused into the row DCT-II, d += alpha p is paid by
    the row DCT-III pass: the fused update reads q, r and writes r, T1; the
    last pass reads T, p_old, d and writes p, d."""
    N = M = 8192
    px = N * M
    launches = [("stencil", 0.2), ("alpha", 0.005), ("update_dct2", 0.2), ("transpose", 0.05),
                ("cols", 0.14), ("partials", 0.008), ("transpose", 0.05), ("rows_dct3", 0.17)]
    kern = bench.kernel_table(launches, "f16", "fast", N, M, flexible=False)
    assert kern["fct_rows_fwd_cg_kernel"]["bytes_per_launch"] == 14 * px
    assert kern["fct_rows_inv_kernel"]["bytes_per_launch"] == 18 * px
    assert kern["stencil_kernel"]["bytes_per_launch"] == 16 * px


def test_f64_bytes_double():
    kern = bench.kernel_table([("stencil", 1.0), ("axpy", 1.0)], "f64", "folded", 256, 256, False)
    assert kern["stencil_kernel"]["bytes_per_launch"] == 48 * 256 * 256
    assert kern["axpy_kernel"]["bytes_per_launch"] == 48 * 256 * 256


def test_fast_plain_beta_stencil_applies_the_operator_only():
    """Fast form, plain beta: the stencil reads p, Ov, Oh and writes q."""
    kern = bench.kernel_table([("stencil", 1.0), ("rows_dct3", 1.0)], "f16", "fast", 256, 256,
                              False)
    assert kern["stencil_kernel"]["bytes_per_launch"] == 16 * 256 * 256
    assert kern["fct_rows_inv_kernel"]["bytes_per_launch"] == 10 * 256 * 256


def test_roofline_skips_the_issue_bound_column_pass():
    """The column pass is reported as bound by instruction issue and never
    priced against the HBM peak, even where it takes the most time."""
    kern = bench.kernel_table([("stencil", 0.1), ("cols", 0.5), ("rows_dct3", 0.2)], "f16",
                              "fast", 512, 512, False)
    roof = bench.roofline(kern, "f16")
    assert roof["kernel"] == "fct_rows_inv_kernel" and roof["bound"] == "hbm"


def test_alu_roofline_of_the_column_pass():
    """The column pass (bound by instruction issue) is rated in
    lane-instructions per second against 256 CUs x 4 SIMDs x 16 lanes x
    2.4 GHz."""
    kern = {"fct_cols_kernel": {"bound": "alu", "launches": 1, "ms": 0.1, "bytes_per_launch": 1},
            "stencil_kernel": {"bound": "hbm", "launches": 1, "ms": 0.2, "bytes_per_launch": 1}}
    out = bench.alu_roofline(kern, {"fct_cols_kernel": 1e6})
    assert list(out) == ["fct_cols_kernel"]
    ach = 1e6 * 64 / 1e-4 / 1e12
    assert abs(out["fct_cols_kernel"]["achieved"] - ach) < 0.01
    assert abs(bench.VALU_PEAK_T - 39.3216) < 1e-3
