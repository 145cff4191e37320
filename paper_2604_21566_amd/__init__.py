"""MI355X-native large-number add / sub / mul (placeholder; binding added next)."""
