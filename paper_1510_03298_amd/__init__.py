"""MI355X-native l1-penalised GLAM solver (rho-transform chain, GD-PG path).

Importing the package is cheap: the HIP library is loaded by
``paper_1510_03298_amd.glam`` (which raises if the built library is missing).
"""
__all__ = ["inputs"]
