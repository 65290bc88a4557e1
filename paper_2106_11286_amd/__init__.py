"""MI355X-native colour-sweep Metropolis for the anisotropic classical
Heisenberg model (arXiv:2106.11286, Eq. (1)).

``paper_2106_11286_amd.mcheis`` is the Python binding of the HIP library
``libmcheis.so`` (build it with ``python -m paper_2106_11286_amd.build``);
``paper_2106_11286_amd.workloads`` holds the seeded synthetic workloads.
"""
__all__ = ["mcheis", "workloads", "build"]
