"""Seeded synthetic input generators shared by the oracle tests, the parity tests and the benchmark."""
