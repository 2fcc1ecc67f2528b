"""MI355X semi-Lagrangian Monte-Carlo library for drift-diffusion SDEs (arXiv:2009.07340).

The hot path runs in the HIP library ``libsl_mi355x.so`` behind the C ABI of
``include/sl.h``; ``binding`` mirrors that ABI function by function and
``problem.Problem`` wraps one handle for a workload.  ``workloads`` holds the
seeded input generators.
"""
__all__ = ["binding", "problem", "workloads"]
