"""MI355X-native dual-way streaming PARAFAC2 update (DASH) behind a C-ABI library."""
