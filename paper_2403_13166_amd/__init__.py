"""MI355X-native line-segment tracking object builder (MD -> LS -> T3 -> T5 + T5-DNN)."""
