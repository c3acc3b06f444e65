"""FP64 CPU oracle of the split-step z-loop (test infrastructure only)."""
