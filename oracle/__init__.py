"""CPU oracle (test infrastructure only; see spfc_oracle)."""
