"""MI355X-native pseudo-spectral DNS right-hand side (arXiv:2012.04838)."""
