"""MI355X-native GKB / Ine-TSVD / HKT solver for multiquadric-RBF 3D Helmholtz collocation."""
