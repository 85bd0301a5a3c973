"""Oracle for the recursive multibaryon correlator method (test infrastructure only)."""
