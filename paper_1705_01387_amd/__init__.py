"""MI355X-native Chebyshev/KPM linear-scaling Kubo transport path (placeholder, binding follows)."""
