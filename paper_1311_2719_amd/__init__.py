"""stagcg: staggered-fermion D_slash and conjugate-gradient solves on MI355X.

The compute path lives in the HIP library `libstagcg.so` (sources under
`csrc/`, C ABI in `include/stagcg.h`); `binding` marshals arguments to it.
Importing this package loads nothing: the library is opened on first use of
`paper_1311_2719_amd.binding`, and fails loudly if it has not been built.
"""

__all__ = ["binding", "inputs", "build"]
