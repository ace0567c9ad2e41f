"""MI355X-native hybrid micro-macro parareal solver (arXiv:2511.13386).

The compute path is the HIP library ``libsth.so`` behind the C-ABI declared in
``include/sth.h``; :mod:`paper_2511_13386_amd.sth` is its thin ctypes binding.
Importing the package loads nothing; the library is loaded on first use and
the binding raises if it is missing.
"""

__all__ = ["sth", "workloads"]
