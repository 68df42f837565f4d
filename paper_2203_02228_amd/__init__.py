"""FACO (Focused Ant Colony Optimization) hot path for MI355X."""
