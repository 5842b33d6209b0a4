"""libalp: MI355X-native actuator-line coupling operator (package stub)."""
