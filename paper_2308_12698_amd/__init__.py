"""MI355X-native batched quadrotor simulator (hot path of arXiv 2308.12698)."""
