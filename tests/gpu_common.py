"""Shared helpers for the GPU parity tests (HIP path vs the FP64 oracle)."""
import numpy as np

from oracle import ahr_oracle as O


def f32(x):
    return float(np.float32(x))


def params32(p: O.HintParams) -> O.HintParams:
    """The boundary takes float32 parameters; give the oracle the same values."""
    return O.HintParams(p.nbx, p.nby, f32(p.detection_ratio), f32(p.bin_capacity), f32(p.mu), p.clique_max,
                        p.expand_macro_pins, p.macro_hints, p.bin_hints, f32(p.prune_tau))


def spec32(s: O.FilterSpec) -> O.FilterSpec:
    return O.FilterSpec(tuple(s.ks), tuple(f32(a) for a in s.alphas), f32(s.sigma), s.lambda_mode,
                        f32(s.lambda_fixed))


def to_c_params(A, p: O.HintParams):
    flags = ((A.EXPAND_MACRO_PINS if p.expand_macro_pins else 0) | (A.MACRO_HINTS if p.macro_hints else 0)
             | (A.BIN_HINTS if p.bin_hints else 0))
    return A.hint_params(p.nbx, p.nby, p.detection_ratio, p.bin_capacity, p.mu, p.clique_max, flags, p.prune_tau)


def to_c_spec(A, s: O.FilterSpec):
    mode = A.LAMBDA_FIXED if s.lambda_mode == "fixed" else A.LAMBDA_GERSHGORIN
    return A.filter_spec(s.ks, s.alphas, s.sigma, mode, s.lambda_fixed)


def movable_rows(nl):
    return (nl["node_flags"] & O.FLAG_FIXED) == 0


def rel_err(y, ref, rows):
    """Centred relative Frobenius error over the given rows."""
    y = np.asarray(y, np.float64)[rows]
    ref = np.asarray(ref, np.float64)[rows]
    den = np.linalg.norm(ref - ref.mean(axis=0))
    return float(np.linalg.norm(y - ref) / den)


def row_err(y, ref, rows):
    """Largest error of any single element over the given rows, relative to
    the largest centred magnitude of the reference there (a per-row bound
    next to the norm: a few rows off by a site cannot hide in it)."""
    y = np.asarray(y, np.float64)[rows]
    ref = np.asarray(ref, np.float64)[rows]
    scale = np.max(np.abs(ref - ref.mean(axis=0)))
    return float(np.max(np.abs(y - ref)) / scale) if y.size else 0.0


def check_filter(y, ref, rows, tol=1e-5):
    """Filter parity: centred relative Frobenius error and the per-element
    error (row_err) both within tol.  Returns the Frobenius error."""
    rel, row = rel_err(y, ref, rows), row_err(y, ref, rows)
    assert rel <= tol and row <= tol, f"centred rel err {rel:.3e}, max element err {row:.3e} (bound {tol:g})"
    return rel


def sorted_rows(row_ptr, col, val):
    """Entries ordered by (row, col): the canonical order of a CSR."""
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    o = np.lexsort((col, rows))
    return rows[o], np.asarray(col)[o], np.asarray(val)[o]
