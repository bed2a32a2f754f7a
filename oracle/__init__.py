"""CPU oracle of the Gaussian-parameter path (test infrastructure only)."""
