"""Seeded synthetic inputs shared by the tests, the benchmark, the oracle's
golden-value script and the pretraining driver. Holds no method arithmetic."""
