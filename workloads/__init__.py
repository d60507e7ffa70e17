"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws positions, charges, densities, sub-box origins and
quadrature parameters. It holds none of the lattice-summation arithmetic: the
GPU library and the CPU oracle each compute everything else on their own.

Every generator is deterministic in its seed. The five named workloads follow
the paper's synthetic lattices of point charges (hydrogen-like unit charges in
a box, Sec. 3.1; a periodic supercell, Sec. 3.2) at the sizes the benchmark
uses; ``small_*`` generators give oracle-sized cases of the same structure.
"""
from .configs import (System, Density, make_density, rule_s_params, quad_spec,
                      config1, config2, config3, config4, config5,
                      small_box, small_periodic, make_basis, CONFIGS, tensor_coords,
                      small_tensor, config_tensor, config_slab)

__all__ = ["System", "Density", "make_density", "rule_s_params", "quad_spec",
           "config1", "config2", "config3", "config4", "config5",
           "small_box", "small_periodic", "make_basis", "CONFIGS", "tensor_coords",
           "small_tensor", "config_tensor", "config_slab"]
