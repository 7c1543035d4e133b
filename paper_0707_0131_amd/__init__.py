"""eigCG on MI355X: deflated CG for many right-hand sides of the Wilson normal
equations, as a HIP library (libeigcg.so, C ABI in include/eigcg.h) with a
thin ctypes binding.

Method: Stathopoulos and Orginos, arXiv:0707.0131 (eigCG, init-CG and
Incremental eigCG).  Import ``paper_0707_0131_amd.binding`` for the entry
points; it raises ImportError when the library has not been built.
"""

__all__ = ["binding"]
