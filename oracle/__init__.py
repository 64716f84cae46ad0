"""CPU oracle for the stealthy-hyperuniform hot path (test infrastructure only)."""
