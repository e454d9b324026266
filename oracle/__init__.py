"""CPU oracle for the replica-exchange polymer hot path (test infrastructure only)."""
