"""The byte model behind the benchmark's roofline figures (CPU only).

bench.py prices each kernel of a step with the algorithmic bytes of the
survey's per-unit model and divides by the kernel's measured duration.  These
tests pin that model to the closed forms it is defined by: the per-piece
bytes of one evaluation, their sum for a residual and a product, the
Gram-Schmidt bytes of the delayed-reorthogonalisation CGS2 against the
every-column CGS2 figure, and the fractions recomputed from durations.
"""
import math

import pytest

import bench

N, NA, PHI, M = 2048, 4_192_413.0, 1.0, 30


def test_product_pieces_fp32():
    nf = N * N
    assert bench.kernel_bytes("prolong", N, NA, PHI, 4, M) == 4 * nf + 12 * NA
    for p in ("fft_rows", "fft_cols", "fft_rows_inv"):
        assert bench.kernel_bytes(p, N, NA, PHI, 4, M) == 8 * nf
    for phi in (0.25, 0.7246, 1.0):
        assert bench.kernel_bytes("jvp", N, NA, phi, 4, M) == pytest.approx(24 * nf * phi + 12 * NA, rel=1e-15)


def test_one_evaluation_sums_fp32():
    """Pi + three Poisson passes + stencil: (28 + 24 phi_t) N_f + 24 N_a for a
    product and (28 + 8 phi_t) N_f + 24 N_a for a residual, FP32 bulk."""
    nf = N * N
    for phi in (0.3, 1.0):
        jv = sum(bench.kernel_bytes(p, N, NA, phi, 4, M)
                 for p in ("prolong", "fft_rows", "fft_cols", "fft_rows_inv", "jvp"))
        assert jv == pytest.approx((28 + 24 * phi) * nf + 24 * NA, rel=1e-14)
        f = sum(bench.kernel_bytes(p, N, NA, phi, 4, M)
                for p in ("res_prolong", "res_fft_rows", "res_fft_cols", "res_fft_rows_inv", "res_stencil"))
        assert f == pytest.approx((28 + 8 * phi) * nf + 24 * NA, rel=1e-14)


def test_fp64_doubles_the_dense_terms():
    nf = N * N
    for p in ("prolong", "fft_cols", "jvp", "res_stencil"):
        d = bench.kernel_bytes(p, N, NA, 0.5, 8, M) - bench.kernel_bytes(p, N, NA, 0.5, 4, M)
        assert d == pytest.approx(bench.kernel_bytes(p, N, 0.0, 0.5, 4, M), rel=1e-15)
        assert d >= 2 * 0.5 * nf


def test_gram_schmidt_every_column_figure():
    """The every-column CGS2 figure per step, 16 m (m+1) N_a + 64 m N_a, over m
    launches."""
    for m in (1, 12, 20, 30, 47):
        per = bench.kernel_bytes("gram_schmidt", N, NA, PHI, 8, m)
        assert per * m == pytest.approx(16 * m * (m + 1) * NA + 64 * m * NA, rel=1e-15)


def test_delayed_cgs2_reads_half():
    """Column j reads slots 0..j and w once per stage (2 (8 (j + 1) + 8) bytes
    per entry) and writes v_j (j > 0) and r_{j+1} (j < m - 1): summed, half the
    every-column figure less the two writes the first and last columns skip."""
    for m in (1, 2, 20, 30, 47):
        full = 16 * m * (m + 1) + 64 * m
        assert bench.gs_bytes(1.0, m) == full / 2 - 16
        # by enumeration of each column's vectors
        tot = 0
        for j in range(m):
            tot += 2 * (j + 2) * 8 + 8 * ((j > 0) + (j < m - 1))
        assert bench.gs_bytes(1.0, m) == tot


def test_fractions_recompute_from_durations():
    """Achieved bandwidth = algorithmic bytes per launch / average launch time,
    and the RHS pipeline fraction = (B_F + m B_Jv) / (t_F + m t_Jv) / 8 TB/s."""
    prof = {p: 0.0 for p in bench.MODELLED}
    ms = {"res_prolong": 0.065, "res_fft_rows": 0.042, "res_fft_cols": 0.082, "res_fft_rows_inv": 0.085,
          "res_stencil": 0.237, "prolong": 0.050, "fft_rows": 0.0207, "fft_cols": 0.0265, "fft_rows_inv": 0.0217,
          "jvp": 0.086, "gram_schmidt": 0.470}
    for p, t in ms.items():
        prof[p] = t * (M if p in bench.PER_COLUMN else 1)
    k = bench.roofline_from_profile(prof, N, NA, PHI, 2, 4, M)
    nb = bench.kernel_bytes("jvp", N, NA, PHI, 4, M) * 2
    assert k["jvp"]["avg_launch_ms"] == pytest.approx(0.086)
    assert k["jvp"]["achieved_gbs"] == pytest.approx(nb / 0.086e-3 / 1e9)
    assert k["jvp"]["frac"] == pytest.approx(nb / 0.086e-3 / 8e12)
    # the residual phases of an FP32-bulk solve are priced in FP64
    assert k["res_stencil"]["algorithmic_bytes_per_launch"] == pytest.approx(
        2 * (16 * N * N * PHI + 12 * NA))
    r = bench.rhs_pipeline(k, M)
    bf = sum(bench.kernel_bytes(p, N, NA, PHI, 8, M) for p in bench.RESIDUAL) * 2
    bj = sum(bench.kernel_bytes(p, N, NA, PHI, 4, M)
             for p in ("prolong", "fft_rows", "fft_cols", "fft_rows_inv", "jvp")) * 2
    tf = sum(ms[p] for p in bench.RESIDUAL)
    tj = sum(ms[p] for p in ("prolong", "fft_rows", "fft_cols", "fft_rows_inv", "jvp"))
    assert r["frac"] == pytest.approx((bf + M * bj) / ((tf + M * tj) * 1e-3) / 8e12)
    assert 0 < r["frac"] < 1 and math.isfinite(r["frac"])
