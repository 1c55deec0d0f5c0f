"""CPU FP64 oracle (test infrastructure only; see psp_oracle)."""
