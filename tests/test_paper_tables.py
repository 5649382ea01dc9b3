"""The oracle at the paper's own scale against numbers the paper prints.

Example 1 (unit square, P1 on the uniform mesh with h = 1/2048, Dirichlet
boundary eliminated, N = 2047^2 = 4 190 209): Table 1 prints the ratios
lambda_q / lambda_{q+1}.  The oracle's converged eigenvalues of that problem
are stored in tests/golden/oracle_ex1_square2048.txt by
tests/golden/make_fullsize_goldens.py (a full oracle solve takes minutes, so
the run is stored, not repeated here).  The absolute eigenvalues of Table 1
carry a uniform scale factor of about 1 + 6.6e-6 against this discretisation,
so only the ratio columns are compared.  Examples 2 and 3 (Tables 2 and 3)
are compared the same way, through the ratio column and a uniform scale."""
import numpy as np

import pytest

from tests.goldens import oracle_eigenvalues, paper_table1_ratios, paper_table2, paper_table3

# Table 2's eigenvalues carry a scale factor of about 1 + 7.2e-7 against this
# discretisation (as Table 1's carry one of about 1 + 6.6e-6); it drifts by
# 2.6e-11 between q = 1 and q = 30, below the algebraic errors the table's last
# column reports.  So the eigenvalues are compared through lambda_q /
# lambda_q^paper, which must agree across q to 5e-11, and the ratio column
# directly.
TABLE2_SCALE_SPREAD_TOL = 5e-11
TABLE2_SCALE_TOL = 1e-6
TABLE2_RATIO_TOL = 1e-11


def table2_differences(lam):
    """(spread of lambda_q / lambda_q^paper over q, its mean - 1, largest
    difference from the printed ratio column) for eigenvalues lam[0..30]."""
    t = paper_table2()
    scale = np.array([lam[q - 1] / v for q, (v, r) in t.items()])
    ratio_err = max(abs(lam[q - 1] / lam[q] - r) for q, (v, r) in t.items() if r is not None)
    return float(scale.max() - scale.min()), float(scale.mean() - 1.0), float(ratio_err)


def test_oracle_reproduces_table1_ratio_column():
    th, rho, head = oracle_eigenvalues("ex1_square2048")
    assert any("N = 4190209" in h and "q = 14" in h for h in head)
    assert rho[:14].max() <= 2e-9  # converged to the stop rule the file records
    ratios = paper_table1_ratios()
    assert sorted(ratios) == [1, 3, 4, 6, 8, 10, 11, 13]
    diff = np.array([abs(th[q - 1] / th[q] - r) for q, r in ratios.items()])
    assert diff.max() < 1e-11, diff
    # ascending, and the pairs the paper prints without a ratio (q = 2, 5, 7, 9,
    # 12) are near-degenerate: the ratio after them is omitted because
    # lambda_q ~ lambda_{q+1}
    assert np.all(np.diff(th[:14]) > 0)
    for q in (2, 5, 7, 9, 12):
        assert th[q] / th[q - 1] - 1 < 1e-5


def test_table2_fixture_is_self_consistent():
    """Each ratio printed in Table 2 is the quotient of the printed eigenvalues
    (guards the transcription in tests/golden/paper_table2.txt)."""
    t = paper_table2()
    assert sorted(t) == list(range(1, 31))
    for q, (lam, r) in t.items():
        if r is not None and q + 1 in t:
            assert abs(lam / t[q + 1][0] - r) < 1e-15, q
    assert all(t[q][0] < t[q + 1][0] for q in range(1, 30))


def test_oracle_reproduces_table2():
    """Example 2 (L-shape, h = 1/1024, N = 2047^2 - 1024^2): the stored oracle
    run reproduces Table 2's eigenvalues (up to the uniform scale) and its
    ratio column."""
    g = oracle_eigenvalues("ex2_lshape1024")
    if g is None:
        pytest.skip("tests/golden/oracle_ex2_lshape1024.txt not written")
    th, rho, head = g
    assert any("N = 3141633" in h and "q = 31" in h for h in head)
    assert rho[:31].max() <= 2e-9
    spread, scale, ratio_err = table2_differences(th)
    assert spread < TABLE2_SCALE_SPREAD_TOL and abs(scale) < TABLE2_SCALE_TOL, (spread, scale)
    assert ratio_err < TABLE2_RATIO_TOL, ratio_err


# Example 3 (-div(K grad u) on (-1,1)^2 with K = 1e3 / 1e-3 / 1 by quadrant,
# h = 1/1024): the coefficient contrast of 1e6 puts the FP64 floor of the
# relative residual near rho = 1e-6, so the stored run stops at rho <= 2e-6
# (STORED_RHO_EX3).  The oracle forms the projected pencil (3.3) literally and
# reduces it through the eigen-decomposition of M^; at that floor this leaves
# its eigenvalues 1e-7 - 3e-7 from Table 3 (ratios within 1.25e-7, with
# Gauss-Seidel smoothing as with Chebyshev), while the library's
# M-orthonormal form of the same pencil reproduces the table to 1.1e-11 in
# its ratios and to one scale factor constant to 8e-11 (the GPU test).  So
# the oracle is held to Table 3 at its own level and the GPU at the table's.
STORED_RHO_EX3 = 2e-6
ORACLE_TABLE3_SPREAD_TOL = 5e-7
ORACLE_TABLE3_RATIO_TOL = 2e-7
TABLE3_SCALE_SPREAD_TOL = 2e-10
TABLE3_SCALE_TOL = 1e-6
TABLE3_RATIO_TOL = 2e-11
EX3_ORACLE_TOL = 1e-6  # GPU against the stored oracle run: the oracle's accuracy here


def table3_differences(lam):
    """(spread of lambda_q / lambda_q^paper over q, its mean - 1, largest
    difference from the printed ratio column) for eigenvalues lam[0..30]."""
    t = paper_table3()
    scale = np.array([lam[q - 1] / v for q, (v, r) in t.items()])
    ratio_err = max(abs(lam[q - 1] / lam[q] - r) for q, (v, r) in t.items() if r is not None)
    return float(scale.max() - scale.min()), float(scale.mean() - 1.0), float(ratio_err)


def test_table3_fixture_is_self_consistent():
    """Each ratio printed in Table 3 is the quotient of the printed eigenvalues
    (guards the transcription in tests/golden/paper_table3.txt)."""
    t = paper_table3()
    assert sorted(t) == list(range(1, 31))
    for q, (lam, r) in t.items():
        if r is not None and q + 1 in t:
            assert abs(lam / t[q + 1][0] - r) < 1e-15, q
    assert all(t[q][0] < t[q + 1][0] for q in range(1, 30))
    # the pairs printed without a ratio nearly coincide
    for q, (lam, r) in t.items():
        if r is None:
            assert t[q + 1][0] / lam - 1 < 3e-5, q


def test_oracle_reproduces_table3():
    """Example 3 (N = 2047^2): the stored oracle run reproduces Table 3's
    eigenvalues (up to the uniform scale) and its ratio column, to the
    accuracy its literal projected pencil reaches at this contrast."""
    g = oracle_eigenvalues("ex3_quadrants1024")
    if g is None:
        pytest.skip("tests/golden/oracle_ex3_quadrants1024.txt not written")
    th, rho, head = g
    assert any("N = 4190209" in h and "q = 31" in h for h in head)
    assert rho[:31].max() <= STORED_RHO_EX3
    spread, scale, ratio_err = table3_differences(th)
    assert spread < ORACLE_TABLE3_SPREAD_TOL and abs(scale) < TABLE3_SCALE_TOL, (spread, scale)
    assert ratio_err < ORACLE_TABLE3_RATIO_TOL, ratio_err
