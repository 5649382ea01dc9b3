"""Readers of the stored reference values under tests/golden/ (the paper's
printed numbers, and eigenvalues written by the oracle's full-size runs)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_table1_ratios():
    """{q: lambda_q / lambda_{q+1}} as printed in Table 1 (Example 1)."""
    out = {}
    for line in open(os.path.join(GOLDEN, "paper_table1_ratios.txt")):
        if line.strip() and not line.startswith("#"):
            q, r = line.split()
            out[int(q)] = float(r)
    return out


def paper_table2():
    """{q: (lambda_q, lambda_q / lambda_{q+1} or None)} as printed in Table 2
    (Example 2); None where the table leaves the ratio blank."""
    out = {}
    for line in open(os.path.join(GOLDEN, "paper_table2.txt")):
        if line.strip() and not line.startswith("#"):
            q, lam, r = line.split()
            out[int(q)] = (float(lam), None if r == "-" else float(r))
    return out


def paper_table3():
    """{q: (lambda_q, lambda_q / lambda_{q+1} or None)} as printed in Table 3
    (Example 3); None where the table leaves the ratio blank."""
    out = {}
    for line in open(os.path.join(GOLDEN, "paper_table3.txt")):
        if line.strip() and not line.startswith("#"):
            q, lam, r = line.split()
            out[int(q)] = (float(lam), None if r == "-" else float(r))
    return out


def oracle_eigenvalues(name):
    """(theta[qe], rho[qe], header lines) of tests/golden/oracle_<name>.txt, or
    None when that file has not been written."""
    path = os.path.join(GOLDEN, "oracle_%s.txt" % name)
    if not os.path.exists(path):
        return None
    th, rho, head = [], [], []
    for line in open(path):
        if line.startswith("#"):
            head.append(line[1:].strip())
        elif line.strip():
            _, t, r = line.split()
            th.append(float(t))
            rho.append(float(r))
    return np.array(th), np.array(rho), head
