"""MI355X-native differentiable vertex model (periodic 2-D epithelia)."""
