"""FP64 CPU oracle of the fully discrete Lax--Oleinik scheme (test infrastructure only)."""
