"""MI355X-native IFGF operator library (Bauinger and Bruno, arXiv 2010.02857)."""
