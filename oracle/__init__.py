"""FP64 CPU oracle for the NCL KKT hot path (test infrastructure only)."""
