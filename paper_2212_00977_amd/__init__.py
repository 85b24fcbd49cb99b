"""MI355X-native SPC 2-hop label index (PSPC round-by-distance PULL build + query)."""
