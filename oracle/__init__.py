"""CPU FP64 oracle (test infrastructure only; see lbpf_oracle.c)."""
