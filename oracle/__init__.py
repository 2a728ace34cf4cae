"""CPU FP64 reference implementation (test infrastructure only; see gp_oracle)."""
