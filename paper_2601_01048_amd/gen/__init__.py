"""IR builder and seeded synthetic workloads (inputs only, no checking arithmetic)."""
