"""MI355X-native explicit step of the 3D crack element method (ES-T-FEM on
linear tetrahedra with split crack elements)."""
