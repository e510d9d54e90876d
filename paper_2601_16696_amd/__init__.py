"""MI355X-native hot path of the Late Adjusted Parallel Sampler (LAPS, arXiv 2601.16696)."""
