"""FSZ on MI355X: error-bounded lossy compression of float32 fields."""
