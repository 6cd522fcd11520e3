"""MI355X-native unbounded (free-space) Poisson solver: Python binding of the
``libups`` C-ABI library (see include/ups.h).

The HIP library is loaded on first use; importing the package alone (e.g. for
``workloads``) does not need it.
"""
