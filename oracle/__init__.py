"""FP64 CPU oracle for the HSGD refinement step (test infrastructure; see hsgd_oracle)."""
