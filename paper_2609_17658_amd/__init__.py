"""MI355X-native short-range TreePM tree force (octree build + group walk)."""
