"""CPU FP64 oracle (test infrastructure only; see lobpcg_oracle)."""
