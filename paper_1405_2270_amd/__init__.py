"""latsum for MI355X: assembled canonical-tensor lattice sums of Newton potentials.

Hot path (Khoromskaia & Khoromskij, arXiv 1405.2270): quadrature table ->
kernel vectors -> lattice assembly -> energy / reconstruction, plus forces by
the adjoint. All arithmetic runs in the HIP library ``liblatsum.so``; this
package only marshals torch tensors into its C ABI.
"""
from .api import (LatticeSpec, TensorLatticeSpec, QuadTable, quadrature, master_halfwidth,
                  kernel_vectors, assemble, assemble_into, assemble_tensor,
                  reconstruct, reconstruct_into, reconstruct_prepare, reconstruct_tiles,
                  reconstruct_autotune, reconstruct_tuned_tile, reconstruct_f16_plan, energy, forces,
                  LatticeEnergy,
                  lattice_energy, Batch, batch_cache_file, combine, richardson,
                  nuclear_matrix, qtt_compress, qtt_expand, probe_copy, probe_mfma)

__all__ = ["LatticeSpec", "TensorLatticeSpec", "QuadTable", "quadrature", "master_halfwidth",
           "kernel_vectors", "assemble", "assemble_into", "assemble_tensor", "reconstruct", "reconstruct_into", "reconstruct_prepare",
           "reconstruct_tiles", "reconstruct_autotune", "reconstruct_tuned_tile", "reconstruct_f16_plan", "energy", "forces",
           "LatticeEnergy", "lattice_energy", "Batch", "batch_cache_file", "combine", "richardson",
           "nuclear_matrix", "qtt_compress", "qtt_expand", "probe_copy", "probe_mfma"]
