"""MI355X-native EDFFS hybrid-GA hot path (arXiv 1903.10741).

The compute path is the HIP library ``libffsga.so`` behind the C ABI in
``include/ffsga.h``; ``paper_1903_10741_amd.ffsga`` is its Python binding
(argument marshalling only). ``paper_1903_10741_amd.workloads`` draws the
seeded synthetic inputs. Importing this package loads nothing.
"""
