"""Block-wise singular value decomposition with a global truncation, and the
block-wise eigen (spectral) and polar decompositions (oracle; test
infrastructure only).

A symmetric matrix is block diagonal in its sectors, so its SVD is the SVD
of each degeneracy matrix on its own (section "Factorization of a matrix";
eq:svd0, eq:svd1): T = (+)_s T_s (x) I_{w_s} with T_s = U_s S_s V_s, and the
singular values of the whole matrix are those of every T_s, each repeated
w_s times (w_s = 1 for the Abelian groups, 2e + 1 for the SU(2) sector of
coupled spin e).  Truncating the whole matrix to its largest values is then
a cut over all sectors' values counted with those multiplicities.

The thesis obtains the spectral and polar decompositions the same way, one
block at a time: here the eigenvalues of each sector's symmetric part, and
the polar factors W = U Vt and P = V diag(s) Vt (or U diag(s) U^T) of each
sector from numpy's SVD.

Sector matrices are built here from the canonical block list directly: rows
are the label tuples of the first n_row legs (with the internal spin for
SU(2)), columns those of the remaining legs, each tuple's degeneracy indices
row-major.  Singular values do not depend on the order of rows or columns
inside a sector, so no layout has to agree with the library's.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from . import tensors as T


def _row_charge(spec, labels, n_row):
    s = sum(q if spec.legs[i].arrow == T.IN else -q for i, q in enumerate(labels[:n_row])) \
        if spec.group != T.U1xU1 else \
        tuple(sum(q[c] if spec.legs[i].arrow == T.IN else -q[c] for i, q in enumerate(labels[:n_row]))
              for c in range(2))
    if spec.group in (T.Z2, T.Z2F):
        s %= 2
    return s


def sector_matrices(spec, flat, n_row: int) -> Dict[object, np.ndarray]:
    """{sector: FP64 matrix} of a tensor split after its first n_row legs.
    Abelian sector = charge flowing in through the row legs; SU(2) (n_row = 2
    on the OPERATOR or LEFT tree) sector = the intermediate spin."""
    blocks = T.split_flat(spec, np.asarray(flat, dtype=np.float64))
    rows: Dict[object, Dict[tuple, int]] = {}
    cols: Dict[object, Dict[tuple, int]] = {}
    shapes = {}
    for (lab, e), blk in blocks.items():
        sec = e if spec.group == T.SU2 else _row_charge(spec, lab, n_row)
        rt, ct = lab[:n_row], lab[n_row:]
        rows.setdefault(sec, {})[rt] = int(np.prod(blk.shape[:n_row], dtype=np.int64))
        cols.setdefault(sec, {})[ct] = int(np.prod(blk.shape[n_row:], dtype=np.int64))
        shapes[(lab, e)] = blk.shape
    out = {}
    for sec in rows:
        roff, r = {}, 0
        for t in sorted(rows[sec]):
            roff[t] = r
            r += rows[sec][t]
        coff, c = {}, 0
        for t in sorted(cols[sec]):
            coff[t] = c
            c += cols[sec][t]
        m = np.zeros((r, c))
        for (lab, e), blk in blocks.items():
            if (e if spec.group == T.SU2 else _row_charge(spec, lab, n_row)) != sec:
                continue
            rt, ct = lab[:n_row], lab[n_row:]
            m[roff[rt]:roff[rt] + rows[sec][rt], coff[ct]:coff[ct] + cols[sec][ct]] = \
                blk.reshape(rows[sec][rt], cols[sec][ct])
        out[sec] = m
    return out


def block_singular_values(spec, flat, n_row: int) -> Dict[object, np.ndarray]:
    """{sector: singular values, descending} by numpy's SVD of each sector matrix."""
    return {s: np.linalg.svd(m, compute_uv=False) for s, m in sector_matrices(spec, flat, n_row).items()}


def symmetric_eigenvalues(m: np.ndarray) -> np.ndarray:
    """Eigenvalues, descending, of the symmetric part (m + m^T) / 2 of a square
    matrix (numpy's symmetric eigensolver)."""
    m = np.asarray(m, dtype=np.float64)
    if m.ndim != 2 or m.shape[0] != m.shape[1]:
        raise ValueError("the symmetric part needs a square matrix")
    return np.linalg.eigvalsh(0.5 * (m + m.T))[::-1]


def block_eigenvalues(spec, flat, n_row: int) -> Dict[object, np.ndarray]:
    """{sector: eigenvalues, descending} of the symmetric part of each sector
    matrix: the block-wise eigen-decomposition, the same per-sector
    factorisation as the SVD's (section "Factorization of a matrix").  Row i
    and column i of a sector are the same label tuple and degeneracy index
    when the column legs repeat the row legs' spectra, which is when the
    symmetric part describes an operator."""
    return {s: symmetric_eigenvalues(m) for s, m in sector_matrices(spec, flat, n_row).items()}


def polar_factors(m: np.ndarray):
    """(W, P) of the polar decomposition of a matrix from numpy's SVD
    m = U diag(s) Vt: W = U Vt, and P = V diag(s) Vt with m = W P when
    rows >= columns, else P = U diag(s) U^T with m = P W."""
    m = np.asarray(m, dtype=np.float64)
    u, sv, vt = np.linalg.svd(m, full_matrices=False)
    w = u @ vt
    p = (vt.T * sv) @ vt if m.shape[0] >= m.shape[1] else (u * sv) @ u.T
    return w, p


def block_polar(spec, flat, n_row: int) -> Dict[object, tuple]:
    """{sector: (W, P)} of each sector matrix (section "Factorization of a
    matrix": the polar decomposition, like the SVD, is taken block by
    block)."""
    return {s: polar_factors(m) for s, m in sector_matrices(spec, flat, n_row).items()}


def multiplicity(spec, sector) -> int:
    return sector + 1 if spec.group == T.SU2 else 1


def truncate(spec, values: Dict[object, np.ndarray], chi_max: int, tol: float = 0.0) -> Tuple[Dict[object, int], float]:
    """Keep the largest singular values over all sectors, each counting
    multiplicity(sector) towards chi_max, stopping at the first value that
    does not fit (or is not above tol).  Returns ({sector: kept}, the sum of
    multiplicity * s^2 over the dropped values)."""
    items: List[Tuple[float, object]] = []
    for s, v in values.items():
        items += [(float(x), s) for x in v]
    items.sort(key=lambda it: -it[0])
    keep = {s: 0 for s in values}
    used, lost, open_ = 0, 0.0, True
    for x, s in items:
        w = multiplicity(spec, s)
        if open_ and x > tol and used + w <= chi_max:
            used += w
            keep[s] += 1
        else:
            open_ = False
            lost += w * x * x
    return keep, lost
