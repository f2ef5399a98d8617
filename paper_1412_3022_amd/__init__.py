"""MI355X-native product-matrix regenerating codes (GF(2^8) region matrix engine)."""
