"""Plain CPU oracle for the RANMAR hot path (test infrastructure only)."""
