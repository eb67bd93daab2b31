"""FP64 CPU oracle for spaND (test infrastructure only; see spand_oracle)."""
