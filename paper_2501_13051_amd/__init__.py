"""MI355X-native semi-naive Datalog engine over column-stored uint32 relations.

The engine itself is the C-ABI library libfv.so (HIP kernels for gfx950 and
a C++ host runtime, sources in csrc/, declarations in include/fv.h).  This
package holds the thin ctypes binding (`fv`) and the seeded workload
generators (`workloads`).  Importing the package loads nothing native; the
binding loads libfv.so on first use and raises if it has not been built.
"""
__all__ = ["fv", "workloads"]
