"""MI355X-native recursive sweeping preconditioner for the 3D Helmholtz equation."""
