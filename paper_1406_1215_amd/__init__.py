"""MI355X-native Chung-Lu edge generator (Alam & Khan, arXiv:1406.1215)."""
