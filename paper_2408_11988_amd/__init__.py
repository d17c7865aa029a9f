"""TS-SpGEMM on AMD Instinct MI355X (gfx950).

C = A B with A a square n x n sparse matrix and B a sparse n x d tall-and-skinny
matrix (Sec. II-A of "Distributed-Memory Parallel Algorithms for Sparse Matrix
and Sparse Tall-and-Skinny Matrix Multiplication", SC'24), over plus-times or
the (AND, OR) semiring with a complement mask (multi-source BFS, Sec. IV-A).

This package is a thin binding of the C-ABI library ``libtsspgemm.so``
(``include/tsspgemm.h``): torch supplies device memory and the current HIP
stream; every step of the computation runs in the library's HIP kernels.
"""
from .api import (  # noqa: F401
    DeviceCsr,
    Plan,
    TSSpGEMMError,
    TSSpGEMMFunction,
    TSSpGEMMOp,
    backward,
    bitmap_words,
    column_slice,
    embed_epoch,
    grad_a,
    grad_b,
    masked_bool,
    merge_rows,
    msbfs,
    numeric,
    spgemm,
    spmm,
    spmm_noalloc,
    symbolic,
    tile_edges,
    tiled_spgemm,
    transpose,
    version,
)
