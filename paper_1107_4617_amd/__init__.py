"""Shiftable-kernel (constant-time) bilateral filtering on MI355X (gfx950)."""
