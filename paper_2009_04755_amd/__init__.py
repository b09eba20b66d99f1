"""MI355X-native all-pairs hot path (Rocket, arXiv 2009.04755) -- placeholder, filled in below."""
