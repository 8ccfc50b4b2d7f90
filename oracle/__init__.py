"""CPU FP64 FEAST oracle: test infrastructure only (see feast_oracle)."""
