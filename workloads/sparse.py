"""Seeded sparse bag-of-words matrices standing in for the paper's text
corpora (documents x words, entries are word counts): word frequencies
follow a Zipf law, document lengths a log-normal law.  Returns the matrix in
compressed sparse columns (and rows); holds no arithmetic of the method."""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class SparseMatrix:
    n: int
    p: int
    col_ptr: np.ndarray   # int64, p + 1
    row_idx: np.ndarray   # int32, nnz (ascending within each column)
    col_val: np.ndarray   # float32, nnz
    row_ptr: np.ndarray   # int64, n + 1
    col_idx: np.ndarray   # int32, nnz (ascending within each row)
    row_val: np.ndarray   # float32, nnz

    @property
    def nnz(self):
        return int(self.col_ptr[-1])

    def dense(self):
        """Dense FP64 copy (small matrices only)."""
        A = np.zeros((self.n, self.p))
        cols = np.repeat(np.arange(self.p), np.diff(self.col_ptr))
        A[self.row_idx, cols] = self.col_val
        return A


def bag_of_words(seed, n_docs, n_words, tokens, zipf=1.07, doc_sigma=0.8):
    """`tokens` word draws spread over the documents (log-normal lengths);
    A[d, w] = number of times word w was drawn for document d."""
    rng = np.random.default_rng(seed)
    prob = 1.0 / (np.arange(n_words) + 2.7) ** zipf
    prob /= prob.sum()
    lens = rng.lognormal(0.0, doc_sigma, n_docs)
    lens = np.maximum(1, np.round(lens / lens.sum() * tokens)).astype(np.int64)
    docs = np.repeat(np.arange(n_docs, dtype=np.int64), lens)
    words = rng.choice(n_words, size=docs.size, p=prob).astype(np.int64)
    key, counts = np.unique(words * n_docs + docs, return_counts=True)
    col = key // n_docs
    row = (key % n_docs).astype(np.int32)
    col_ptr = np.zeros(n_words + 1, dtype=np.int64)
    np.cumsum(np.bincount(col, minlength=n_words), out=col_ptr[1:])
    val = counts.astype(np.float32)
    order = np.lexsort((col, row))  # by row, then column
    row_ptr = np.zeros(n_docs + 1, dtype=np.int64)
    np.cumsum(np.bincount(row, minlength=n_docs), out=row_ptr[1:])
    return SparseMatrix(n_docs, n_words, col_ptr, row, val, row_ptr,
                        col[order].astype(np.int32), val[order])
