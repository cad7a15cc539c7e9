"""MI355X-native block-procedural matrix-free product phi = H psi."""
