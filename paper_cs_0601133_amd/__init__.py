"""MI355X-native finite-field matrix multiplication (fgemm)."""
