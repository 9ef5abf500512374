"""CPU oracle (test infrastructure only): see sfac_oracle."""
