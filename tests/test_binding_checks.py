"""Argument checks of the Python binding (CPU only, no library call): a
tensor too short for the N elements the C ABI will read or write, a row
stride below N, or rows past the end of the storage are rejected before any
pointer reaches the library."""
import pytest

torch = pytest.importorskip("torch")

import paper_1707_04950_amd as lib  # noqa: E402


def _c(*shape):
    return torch.zeros(*shape, dtype=torch.complex128)


def test_vector_checks():
    with pytest.raises(ValueError, match="complex128"):
        lib._ptr(torch.zeros(8, dtype=torch.float64), 8)
    with pytest.raises(ValueError, match="needs 8"):
        lib._ptr(_c(7), 8)
    with pytest.raises(ValueError, match="contiguous"):
        lib._ptr(_c(16)[::2], 8)
    # the right size passes the size checks and stops at the device check
    with pytest.raises(ValueError, match="CUDA"):
        lib._ptr(_c(8), 8)
    with pytest.raises(ValueError, match="CUDA"):
        lib._ptr(_c(9), 8)


def test_row_checks():
    with pytest.raises(ValueError, match="2-D"):
        lib._ptr_rows(_c(8), 8)
    with pytest.raises(ValueError, match="needs 8"):
        lib._ptr_rows(_c(3, 7), 8)
    with pytest.raises(ValueError, match="rows"):
        lib._ptr_rows(_c(2, 8), 8, rows=3)
    with pytest.raises(ValueError, match="unit stride"):
        lib._ptr_rows(_c(8, 3).t(), 8)
    # overlapping rows: stride 4 below the row length 8
    base = _c(40)
    with pytest.raises(ValueError, match="row stride"):
        lib._ptr_rows(base.as_strided((3, 8), (4, 1)), 8)
    # a view whose last rows are shorter than N: its span would pass the end
    with pytest.raises(ValueError, match="needs 8"):
        lib._ptr_rows(base.as_strided((3, 6), (8, 1)), 8)
    # padded rows (stride above N) inside the storage pass to the device check
    with pytest.raises(ValueError, match="CUDA"):
        lib._ptr_rows(_c(3, 10)[:, :8], 8)
    with pytest.raises(ValueError, match="CUDA"):
        lib._ptr_rows(_c(3, 8), 8)
