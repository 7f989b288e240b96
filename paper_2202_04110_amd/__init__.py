"""Damped log-domain loopy belief propagation on MI355X (gfx950).

``paper_2202_04110_amd.lbp`` is the binding over the C-ABI library
``liblbp.so`` (HIP kernels); ``workloads`` holds the seeded synthetic graph
generators.  Importing the package loads neither.
"""
