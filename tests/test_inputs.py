"""The seeded input generators: the large selector population stays within
its row range and its entry cap, draws the same matrix for the same index,
and keeps each row's columns sorted and unique (CSR as the library takes
it)."""
import numpy as np
import pytest

from paper_1801_01134_amd import records as R
from paper_1801_01134_amd import synth


def _valid_csr(A):
    assert A.rowptr[0] == 0 and A.rowptr[-1] == A.nnz
    assert np.all(np.diff(A.rowptr) >= 0)
    for i in range(0, A.n_rows, max(1, A.n_rows // 50)):
        cols = A.colidx[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and (cols.size == 0 or (cols[0] >= 0 and cols[-1] < A.n_cols))


@pytest.mark.parametrize("index", range(4))
def test_large_population_respects_rows_and_cap(index, monkeypatch):
    # a small cap, so that the clamp acts on matrices a test can build
    cap = 1 << 16
    monkeypatch.setattr(synth, "LARGE_NNZ_CAP", cap)
    fam, A = synth.large_matrix(index, 3000, 6000)
    assert fam == synth.FAMILIES[index % 4]
    assert 3000 <= A.n_rows <= 6000 and A.n_cols == A.n_rows
    if fam == "powerlaw":
        # not clamped: its mean row length (about 34) keeps 4M rows under 2^28 entries
        assert A.nnz / A.n_rows < 64 and 4_000_000 * 64 < (1 << 28)
    else:
        # the clamp bounds the expected entries per row; the draws may exceed
        # that mean a little, and the diagonal of a banded row is always kept
        assert A.nnz <= 1.25 * cap + A.n_rows, (fam, A.nnz)
    _valid_csr(A)
    fam2, A2 = synth.large_matrix(index, 3000, 6000)
    assert fam2 == fam and np.array_equal(A2.colidx, A.colidx) and np.array_equal(A2.rowptr, A.rowptr)


def test_populations_have_generators():
    for pop in R.POPULATIONS:
        fam, A = R.generator(pop)(1, 2000, 3000)
        assert 2000 <= A.n_rows <= 3000 or pop == "structured"
        _valid_csr(A)


def test_selector_records_span_the_papers_ranges():
    """The generated selector population covers the values per block of the
    paper's test sets (Table 1: Avg(1,8) from 1 to 7.6, Avg(4,8) from 1 to
    30), measured by the device features stored in the committed records."""
    import os
    rec = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1801_01134_amd",
                       "records", "selector_records_mi355x.jsonl")
    if not os.path.exists(rec):
        pytest.skip("no committed records")
    X = np.array([r["features"] for r in R.load(rec)])
    assert X[:, 8].min() <= 1.001 and X[:, 8].max() >= 7.6      # features are FP32
    assert X[:, 12].min() <= 1.001 and X[:, 12].max() >= 30.0
