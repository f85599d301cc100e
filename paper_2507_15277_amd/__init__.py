"""MI355X-native multi-versioned SGEMM with portability-tuned variant sets."""
