"""MI355X-native dynamic-mesh-refinement EM/plasma-fluid library."""
