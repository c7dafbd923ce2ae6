"""FP64 CPU oracle for the compact U(1) multilevel hot path (test infrastructure only)."""
