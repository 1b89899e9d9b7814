"""MI355X-native Stone SIP solver (arXiv:1303.4538 hot path)."""
