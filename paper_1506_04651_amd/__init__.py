"""Batched Radau5 reaction substep for MI355X (gfx950)."""
