"""FP64 CPU oracle (test infrastructure only; see diffcloth_oracle)."""
